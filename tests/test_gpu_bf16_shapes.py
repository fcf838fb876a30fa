"""GPU parity of the bfloat16 hi/lo MFMA power spectrum across shapes,
against the FP64 oracle: one wave per centre with one, two and three row
blocks held in registers (K = 7, 20, 48), four waves per centre just past
that (K = 49) and with a ragged last row block (K = 52), lmax 0 and 12 (one
to seven groups of operand values past 2l+1), and centre counts that leave
the last work-group partly empty.

Seeded N(0, 1) coefficients; the oracle checks a sample of centres (the
first, the last and random ones), a float64 product on the device checks
every centre.  Bound: 2e-3 relative Frobenius error and per centre, as for
the molecules and the 8-species cells."""
import numpy as np
import pytest
import torch

import oracle
import paper_2101_08814_amd as P

from test_gpu_parity import rel, worst_centre

pytestmark = pytest.mark.gpu


def _hypers(S, nmax, lmax):
    return dict(n_species=S, nmax=nmax, lmax=lmax, rcut=5.0, sigma=0.5, cutoff_width=0.5, include_center=1)


@pytest.mark.parametrize("S,nmax,lmax,N", [
    (1, 7, 0, 1001),     # K = 7: one row block, lmax 0
    (2, 10, 12, 515),    # K = 20, lmax 12 (2l+1 = 25): C too large for one wave
    (4, 5, 3, 2050),     # K = 20: two row blocks, the second mostly padding
    (4, 12, 2, 777),     # K = 48: three full row blocks in registers
    (7, 7, 2, 1030),     # K = 49: four waves per centre
    (4, 13, 3, 333),     # K = 52: four waves, ragged last row block
    (8, 16, 8, 600),     # K = 128: more than 64 KB of LDS per work-group
])
def test_bf16_spectrum_shapes_match_oracle(S, nmax, lmax, N):
    hyp = _hypers(S, nmax, lmax)
    K, L2 = S * nmax, (lmax + 1) ** 2
    calc = P.Calculator.from_hypers(hyp)
    rng = np.random.default_rng(4048 + K + lmax)
    c = rng.standard_normal((N, K, L2)).astype(np.float32)
    cd = torch.tensor(c, device="cuda")
    p = calc.power_spectrum(cd, "bf16")
    assert calc.device_status() == 0
    assert p.shape == (N, lmax + 1, K * (K + 1) // 2)
    idx = np.unique(np.concatenate([[0, 1, 2, N - 3, N - 2, N - 1], rng.integers(0, N, 26)]))
    ref = oracle.power_spectrum(hyp, c[idx].astype(np.float64))
    got = p[torch.tensor(idx, device="cuda")].double().cpu().numpy()
    e, w = rel(got, ref), worst_centre(got, ref)
    c64 = cd.double()
    iu = torch.triu_indices(K, K, device="cuda")
    err2 = ref2 = 0.0
    for l in range(lmax + 1):
        cl = c64[:, :, l * l:(l + 1) ** 2].contiguous()
        pl = torch.bmm(cl, cl.transpose(1, 2).contiguous())[:, iu[0], iu[1]]
        d = p[:, l].double() - pl
        err2 += float((d ** 2).sum())
        ref2 += float((pl ** 2).sum())
    e_all = (err2 / ref2) ** 0.5
    print(f"[bf16 spectrum S={S} nmax={nmax} lmax={lmax} N={N}] oracle sample rel={e:.3e} worst centre={w:.3e}, "
          f"all centres rel={e_all:.3e}")
    assert e <= 2e-3 and w <= 2e-3
    assert e_all <= 2e-3
