"""Independent solves on separate contexts (own stream, own matrix handle,
own host thread) run at the same time and give bit-identical results to the
same solves run one after another: the library keeps no shared mutable state
and its reductions are deterministic."""
import sys
import threading

import numpy as np
import pytest

import inputs as I

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_concurrent_solves_match_sequential():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1504_04395_amd as P
    P.load_library()
    A_ = I.convdiff3d(24, (30.0, 20.0, 10.0))
    B = torch.from_numpy(I.gaussian_block(A_.n, 16, seed=0)).cuda()
    methods = ("bl_bicg_rq", "egl_qmr", "bl_bicgstab_rq")
    lanes = {}
    for m in methods:
        st = torch.cuda.Stream()
        c = P.Context(0, stream=st.cuda_stream)
        lanes[m] = (c, P.Matrix.from_csr(c, A_), st)
    seq = {}
    for m in methods:
        c, A, _ = lanes[m]
        X, info = P.solve(c, A, B, m, tol=1e-8, maxit=600)
        seq[m] = (X.cpu().numpy(), info.iterations, info.history.copy())
    par, errors = {}, {}

    def run(m):
        try:
            c, A, _ = lanes[m]
            X, info = P.solve(c, A, B, m, tol=1e-8, maxit=600)
            par[m] = (X.cpu().numpy(), info.iterations, info.history.copy())
        except Exception as ex:
            errors[m] = ex

    for rep in range(2):
        ths = [threading.Thread(target=run, args=(m,)) for m in methods]
        for t in ths:
            t.start()
        for t in ths:
            t.join()
        assert not errors, errors
        for m in methods:
            say(f"rep {rep} {m}: it {par[m][1]} (sequential {seq[m][1]})")
            assert par[m][1] == seq[m][1]
            assert np.array_equal(par[m][0], seq[m][0])
            assert np.array_equal(par[m][2], seq[m][2])
    for c, A, _ in lanes.values():
        A.close()
        c.close()
