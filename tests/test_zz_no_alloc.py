"""GPU: the allocation-free thin QR (skr_block_qr_noalloc, static scratch)
against skr_block_qr, the entry point it mirrors, through the C ABI.

Two calls in a row on one context, the second with a smaller block, each
compared with skr_block_qr on the same input: the same kernels run in the same
launch configuration, so Q and C must agree to the bit; Q is also checked for
orthonormal columns and Q C = Z.  Sizes beyond the static scratch are refused."""
import sys

import numpy as np
import pytest

import inputs as I

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1504_04395_amd as P
    ctx = P.Context(0)
    yield P, ctx
    ctx.close()


@pytest.mark.parametrize("kind", ["real", "complex"])
def test_noalloc_qr_matches_block_qr_twice(env, kind):
    import torch
    P, ctx = env
    cplx = kind == "complex"
    for n, s in ((200_003, 16), (5_001, 7)):            # second call: smaller input
        say(f"noalloc qr {kind} n={n} s={s}")
        Zh = I.gaussian_block(n, s, seed=n + s, complex_=cplx)
        Z = torch.from_numpy(Zh).cuda()
        Qa = torch.empty_like(Z)
        Ca, rc_a = P.block_qr_noalloc(ctx, Z, Qa)
        Qr, Cr, rc_r = P.block_qr(ctx, Z)
        torch.cuda.synchronize()
        Qa = Qa.cpu().numpy()
        Qr = Qr.cpu().numpy()
        assert rc_a == rc_r == 0
        assert np.array_equal(Qa, Qr) and np.array_equal(Ca, Cr)
        np.testing.assert_allclose(Qa.conj().T @ Qa, np.eye(s), atol=1e-13)
        np.testing.assert_allclose(Qa @ Ca, Zh, atol=1e-12 * np.abs(Zh).max())
        assert np.allclose(np.tril(Ca, -1), 0) and np.all(np.real(np.diag(Ca)) > 0)


def test_noalloc_qr_in_place(env):
    import torch
    P, ctx = env
    Zh = I.gaussian_block(3000, 5, seed=4)
    Z = torch.from_numpy(Zh).cuda()
    Qr, Cr, _ = P.block_qr(ctx, Z)
    C, rc = P.block_qr_noalloc(ctx, Z, Z)                 # Q = Z: in place
    torch.cuda.synchronize()
    assert rc == 0 and np.array_equal(Z.cpu().numpy(), Qr.cpu().numpy()) and np.array_equal(C, Cr)


def test_noalloc_qr_refuses_sizes_beyond_its_scratch(env):
    import torch
    P, ctx = env
    Z = torch.zeros(100, 17, dtype=torch.float64, device="cuda")
    with pytest.raises(P.SkrError, match="s <= 16"):
        P.block_qr_noalloc(ctx, Z, torch.empty_like(Z))
    Z = torch.zeros(3, 4, dtype=torch.float64, device="cuda")   # n < s
    with pytest.raises(P.SkrError, match="s <= n"):
        P.block_qr_noalloc(ctx, Z, torch.empty_like(Z))
