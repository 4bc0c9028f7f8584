"""Occupied-pair screening with localised orbitals on the GPU (occk_far_opts.
pair_thresh; the Conclusion's localised-orbital variant).  The library
carries, per j batch, the i up to the last pair whose bound reaches the
threshold; the oracle evaluates exactly that band of pairs (band_ends from
its own pair bound, band_mask) and nothing else.  Gates: the band ends equal
the oracle's (integer decisions; the thresholds sit well away from every
bound value), FP64 <= 1e-8 and FP32 <= 1e-6 against the oracle (normwise)."""
import numpy as np
import pytest

import workloads
from oracle.fmm import Setup, band_ends, band_mask, far_K as oracle_far_K, pair_bound

from conftest import rel

pytestmark = pytest.mark.gpu


def _clear_tau(B, tau):
    """tau nudged so that no bound value lies within 1e-6 (relative) of it."""
    v = np.sort(B.ravel())
    while True:
        k = np.searchsorted(v, tau)
        near = [v[x] for x in (k - 1, k) if 0 <= x < v.size]
        if all(abs(x - tau) > 1e-6 * tau for x in near):
            return tau
        tau *= 1.01


@pytest.fixture(scope="module")
def chain40():
    wl = workloads.alkane_chain(n_carbon=40, depth=5)
    C = workloads.localized_orbitals(wl.system, 7)
    return wl, C, Setup(wl.system, wl.params)


@pytest.mark.parametrize("tau,jb", [(1e-3, 16), (1e-6, 16), (1e-4, 64)])
def test_screened_K_matches_oracle(chain40, tau, jb):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1708_05353_amd import occk
    wl, C, st = chain40
    n = C.shape[1]
    tau = _clear_tau(pair_bound(st, C), tau)
    print(f"[screen] chain40 nbasis {wl.system.nbasis} nocc {n} tau {tau:.3e} jblock {jb}", flush=True)
    tr = occk.Tree(wl.system, wl.params)
    Cd = torch.from_numpy(C).cuda()
    K = torch.full((wl.system.nbasis, n), np.nan, dtype=torch.float64, device="cuda")
    occk.far_K(tr, Cd, K, jblock=jb, pair_thresh=tau)
    torch.cuda.synchronize()
    carried, jbu, ends = occk.pair_screen_info(tr)
    ref_ends = band_ends(st, C, tau, jbu)
    assert np.array_equal(ends, ref_ends), (ends, ref_ends)
    mask = band_mask(n, jbu, ref_ends)
    # carried (j, i) columns: per batch its j times the i from its first j to its end
    want = sum((min(n, (k + 1) * jbu) - k * jbu) * (int(e) - k * jbu) for k, e in enumerate(ref_ends))
    assert carried == want
    ref = oracle_far_K(st, C, pair_mask=mask)
    errs = {"fp64": rel(K.cpu().numpy(), ref)}
    K32 = torch.zeros_like(K)
    occk.far_K(tr, Cd, K32, jblock=jb, pair_thresh=tau, precision=occk.PREC_FP32)
    torch.cuda.synchronize()
    errs["fp32"] = rel(K32.cpu().numpy(), ref)
    print(f"[screen] jblock {jbu} bands {list(ends)} pairs kept {mask.mean():.3f} "
          f"fp64 {errs['fp64']:.2e} fp32 {errs['fp32']:.2e}", flush=True)
    assert errs["fp64"] <= 1e-8 and errs["fp32"] <= 1e-6, errs
    tr.free()


def test_screening_off_equals_unscreened(chain40):
    """pair_thresh = 0 is the unscreened call, bit for bit; a threshold that
    keeps every pair reproduces it to rounding."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1708_05353_amd import occk
    wl, C, st = chain40
    tr = occk.Tree(wl.system, wl.params)
    Cd = torch.from_numpy(C).cuda()
    K0 = torch.zeros((wl.system.nbasis, C.shape[1]), dtype=torch.float64, device="cuda")
    K1 = torch.zeros_like(K0)
    occk.far_K(tr, Cd, K0, jblock=16)
    occk.far_K(tr, Cd, K1, jblock=16, pair_thresh=1e-300)
    torch.cuda.synchronize()
    carried, jbu, ends = occk.pair_screen_info(tr)
    assert np.all(ends == C.shape[1])
    assert rel(K1.cpu().numpy(), K0.cpu().numpy()) <= 1e-14
    tr.free()


def test_alkane_full_size_screened():
    """The 400-carbon chain (nbasis 9610, nocc 1601, L = 2) with localised
    orbitals: the band ends equal the oracle's, the screened K differs from
    the unscreened K (both on the GPU, FP64) by less than the threshold, and
    the band carries a small share of the columns."""
    import time

    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1708_05353_amd import occk
    wl = workloads.alkane_chain()
    C = workloads.localized_orbitals(wl.system, 2)
    st = Setup(wl.system, wl.params, workers=8)
    n = C.shape[1]
    tau = _clear_tau(pair_bound(st, C), 1e-6)
    print(f"[screen] alkane nbasis {wl.system.nbasis} nocc {n} tau {tau:.3e}", flush=True)
    tr = occk.Tree(wl.system, wl.params)
    Cd = torch.from_numpy(C).cuda()
    K0 = torch.zeros((wl.system.nbasis, n), dtype=torch.float64, device="cuda")
    K1 = torch.zeros_like(K0)
    occk.far_K(tr, Cd, K0)
    occk.far_K(tr, Cd, K1, jblock=64, pair_thresh=tau)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    occk.far_K(tr, Cd, K0)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    occk.far_K(tr, Cd, K1, jblock=64, pair_thresh=tau)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    carried, jbu, ends = occk.pair_screen_info(tr)
    assert jbu == 64
    assert np.array_equal(ends, band_ends(st, C, tau, 64))
    share = carried / (n * (n + 1) / 2)
    err = rel(K1.cpu().numpy(), K0.cpu().numpy())
    print(f"[screen] alkane jblock {jbu} carried {carried} ({share:.3f} of the symmetric columns) "
          f"screened-vs-full {err:.2e}; {1e3 * (t1 - t0):.1f} ms full, {1e3 * (t2 - t1):.1f} ms screened",
          flush=True)
    assert err < tau
    assert share < 0.25
    tr.free()
