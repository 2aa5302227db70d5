"""The allocation-free eigendecomposition (kot_eigh_noalloc, a static scratch array per device) against the
context-based kot_eigh, through the C-ABI: two calls in a row, the second with a smaller matrix."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def _n(t):
    return t.detach().cpu().numpy()


def test_noalloc_eigh_matches_kot_eigh(gpu_ctx):
    import torch
    from paper_2310_14087_amd import kotssn
    prm = kotssn.default_params()
    for l in (400, 123):
        print(f"[case] kot_eigh_noalloc random symmetric l={l}", flush=True)
        rng = np.random.default_rng(900 + l)
        A = rng.standard_normal((l, l))
        Z = A + A.T
        Zd = _t(Z)
        P = torch.empty_like(Zd)
        w = torch.empty(l, device="cuda:0", dtype=torch.float64)
        w1, P1 = kotssn.eigh_noalloc(Zd, prm, P=P, w=w)
        torch.cuda.synchronize()
        w0, P0 = gpu_ctx.eigh(Zd, prm)
        w0, P0, w1, P1 = _n(w0), _n(P0), _n(w1), _n(P1)
        scale = np.abs(w0).max()
        assert np.all(np.diff(w1) >= 0)
        np.testing.assert_allclose(w1, w0, atol=1e-13 * scale * l ** 0.5)
        np.testing.assert_allclose(w1, np.linalg.eigvalsh(Z), atol=1e-13 * scale * l ** 0.5)
        assert np.abs(Z @ P1 - P1 * w1).max() <= 1e-13 * scale * l ** 0.5
        assert np.abs(P1.T @ P1 - np.eye(l)).max() <= 1e-13 * l ** 0.5
        # distinct eigenvalues: the same eigenvectors up to sign
        assert np.abs(np.abs(np.sum(P0 * P1, axis=0)) - 1.0).max() <= 1e-9


def test_noalloc_eigh_rejects_oversized_input(gpu_ctx):
    import torch
    from paper_2310_14087_amd import kotssn
    print("[case] kot_eigh_noalloc rejects l=513", flush=True)
    Z = torch.zeros((513, 513), dtype=torch.float64, device="cuda:0")
    with pytest.raises(kotssn.KotError) as e:
        kotssn.eigh_noalloc(Z, kotssn.default_params())
    assert e.value.status == kotssn.KOT_ERR_ARG and "512" in str(e.value)
