"""The operator entry point that allocates nothing (static device scratch),
through the C ABI, against the workspace entry point on the same inputs."""
import numpy as np
import pytest
import torch

from oracle import fwi_oracle as O
from paper_2604_15796_amd import workloads as W

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


@pytest.fixture(scope="module")
def F():
    from paper_2604_15796_amd import fwi
    return fwi


@pytest.fixture(scope="module")
def ctx(F):
    c = F.Context(0)
    yield c
    c.close()


def _dev(x, dtype=torch.complex128):
    return torch.as_tensor(np.ascontiguousarray(x)).to(dtype).to(DEV)


def test_static_scratch_operator_matches_workspace_operator(ctx, F):
    """Two calls in a row, the second on a smaller input (fewer vectors, then
    a smaller 3D grid), in both precisions: the same result as
    fwi_apply_operator bit for bit, and the oracle's operator at the
    operator bar. A problem without cached spectra and a request beyond the
    static scratch are refused with their error codes."""
    p = W.small2d(seed=71, nx=40, nz=33, ne=3, nf=2)
    q = W.small3d(seed=72, nx=12, ny=10, nz=9, ne=3, nf=1)
    for prob, B in ((p, 5), (p, 2), (q, 3), (q, 1)):
        m = O.contrast(prob.c, prob.alpha, prob.c0)
        ctx.green_spectrum(prob, 0)  # spectra cached (allocating call, outside)
        fi = [b % prob.nf for b in range(B)]
        x = W.random_complex(73 + B, (B, prob.n))
        for prec in (0, 1):
            dt = torch.complex64 if prec else torch.complex128
            xd = _dev(x, dt)
            y_ws = ctx.apply_operator(prob, _dev(m), fi, xd, precision=prec)
            y_st = ctx.apply_operator_noalloc(prob, _dev(m), fi, xd, precision=prec)
            assert torch.equal(y_ws, y_st), (prob.name, B, prec)
            y = y_st.cpu().numpy()
            for b in range(B):
                Gh = O.green_spectrum(O.wavenumber(prob.freqs[fi[b]], prob.c0), prob.dim, prob.nx, prob.ny,
                                      prob.nz, prob.dx)
                ref = O.vie_apply(Gh, m, x[b].reshape(prob.shape)).ravel()
                err = np.linalg.norm(y[b] - ref) / np.linalg.norm(ref)
                assert err < (2e-6 if prec else 1e-13), (prob.name, B, prec, err)
    # spectra of another problem are cached now: p is refused
    with pytest.raises(F.FWIError) as e:
        ctx.apply_operator_noalloc(p, _dev(O.contrast(p.c, p.alpha, p.c0)), [0], _dev(np.zeros((1, p.n))))
    assert e.value.code == F.FWI_E_INVAL
    # more scratch than the static array holds: refused, nothing written
    big = W.small3d(seed=74, nx=64, ny=64, nz=64, ne=1, nf=1)
    ctx.green_spectrum(big, 0)
    x = torch.zeros((4, big.n), dtype=torch.complex128, device=DEV)
    with pytest.raises(F.FWIError) as e:
        ctx.apply_operator_noalloc(big, torch.zeros(big.n, dtype=torch.complex128, device=DEV), [0] * 4, x)
    assert e.value.code == F.FWI_E_NOMEM
