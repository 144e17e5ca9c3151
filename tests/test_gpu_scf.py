"""Block-Davidson TC / BITC self-consistent loop of the library (tc_scf), through the C ABI.

* Iterates: the energies of the first iterations equal those of the oracle's block-Davidson loop
  (O5 davidson_scf: the same steps in numpy, with the operator applied as full matrices), with and
  without density-matrix mixing, in TC and BITC mode.
* The 14-electron gas at r_s = 1 from a perturbed start returns to its occupied plane waves: energy
  and orbital energies of the closed forms (O3), in TC and BITC mode.  (At r_s = 2 and 4 the
  plane-wave solution is not a stable fixed point of the loop: small perturbations grow.)
* Small fcc problems: the loop runs to convergence and the oracle checks the fixed point it reached.
  With the library's final orbitals the oracle builds the full matrix of T + h on every k-point's
  plane-wave set (O5).  The orbitals must span an invariant subspace of it (BITC: the right ones a
  right-invariant and the left ones a left-invariant subspace), and its eigenvalues there must be the
  lowest ones.
"""
import numpy as np
import pytest

import tcinputs as T
from oracle import scf as S
from oracle.heg import heg_energy, heg_terms
from oracle.fftroute import MULT

pytestmark = pytest.mark.gpu

tc = pytest.importorskip("paper_2302_07420_amd")


def _say(msg):
    print(msg, flush=True)


def _iterates(w, n, mix=1.0):
    op = tc.from_workload(w, precision=tc.TC_PREC_FP64)
    h, it = op.scf(max_iter=n, pmax=2, etol=1e-300, mix=mix, otol=0.0)
    op.close()
    return h


@pytest.mark.parametrize("case", ["heg2", "heg2_mix", "heg2_bitc", "fcc_nb2"])
def test_iterates_equal_the_oracle_davidson(case):
    heg2 = T.heg_gamma(rs=4.0, nelec=2, grid=8, mmax2=1, occ_m2=0)
    w, n, mix = {
        "heg2": (T.perturbed_start(heg2, 0.4, 3), 6, 1.0),
        "heg2_mix": (T.perturbed_start(heg2, 0.4, 3), 6, 0.5),
        "heg2_bitc": (T.perturbed_start(heg2, 0.4, 3, left_amp=0.3), 6, 1.0),
        "fcc_nb2": (T.tiny_fcc(kmesh=(2, 1, 1), grid=8, ecut=2.0, nb=2, a=6.0, occ=[1.0, 0.7]), 3, 1.0),
    }[case]
    ref, _, _, _ = S.davidson_scf(w, max_iter=n, pmax=2, etol=1e-300, mix=mix)
    got = _iterates(w, n, mix)
    _say(f"[gpu] scf iterates {case}: {list(got)} vs oracle {ref}")
    assert len(got) == len(ref) == n
    np.testing.assert_allclose(got, ref, rtol=1e-11, atol=0)


@pytest.mark.parametrize("amp,left_amp", [(0.5, None), (0.3, 0.2)])
def test_heg14_returns_to_the_closed_forms(amp, left_amp):
    w = T.heg_gamma(rs=1.0)                             # 7 occupied plane waves, 123 in the basis, 16^3
    E0, _ = heg_energy(w)
    eps0, p, f = heg_terms(w)
    lam = sum(MULT.get(t, 1) * e for t, e in eps0.items()) + 0.5 * np.sum(p * p, 1)
    start = T.perturbed_start(w, amp, 17, left_amp=left_amp)
    _say(f"[gpu] scf heg14 from a perturbed start ({'BITC' if left_amp else 'TC'})")
    op = tc.from_workload(start, precision=tc.TC_PREC_FP64)
    E_start = op.energy()[0]
    hist, n = op.scf(max_iter=80, pmax=2, etol=1e-13)
    E = op.energy()[0]
    eps = op.orbital_energies().reshape(-1)
    op.close()
    _say(f"    {n} iterations; E start {E_start:.10f}, end {E:.14f}, closed form {E0:.14f}")
    assert abs(E_start - E0) > 1e-4
    assert n < 80
    assert abs(E - E0) < 1e-10 * abs(E0)
    np.testing.assert_allclose(np.sort(eps.real), np.sort(lam.real), atol=1e-8)


def _fixed_point(w, op, bitc):
    nk = w.nk
    right = [op.get_orbitals(k, left=bitc) for k in range(nk)]
    if bitc:
        R = [r for r, _ in right]
        L = [l for _, l in right]
    else:
        R, L = right, None
    H = S.operator_matrices(w, R, L)
    worst_r = worst_l = worst_e = 0.0
    for k in range(nk):
        Phi = R[k].T                                    # npw x nb
        Hk = H[k]
        if bitc:
            X = L[k].T
            E = X.conj().T @ Hk @ Phi                   # biorthonormal: X^H Phi = 1
            worst_l = max(worst_l, np.abs(X.conj().T @ Hk - E @ X.conj().T).max() / np.abs(Hk).max())
            assert np.abs(X.conj().T @ Phi - np.eye(Phi.shape[1])).max() < 1e-10
        else:
            E = Phi.conj().T @ Hk @ Phi
            assert np.abs(Phi.conj().T @ Phi - np.eye(Phi.shape[1])).max() < 1e-10
        worst_r = max(worst_r, np.abs(Hk @ Phi - Phi @ E).max() / np.abs(Hk).max())
        lam = np.sort(np.linalg.eigvals(Hk).real)
        mine = np.sort(np.linalg.eigvals(E).real)
        worst_e = max(worst_e, np.abs(mine - lam[: len(mine)]).max())
    return worst_r, worst_l, worst_e, R, L


CASES = {
    "tc_k211_g8_nb1": lambda: T.tiny_fcc(kmesh=(2, 1, 1), grid=8, ecut=2.0, nb=1, a=6.0),
    "tc_k211_g8_nb2": lambda: T.tiny_fcc(kmesh=(2, 1, 1), grid=8, ecut=2.0, nb=2, a=6.0, occ=[1.0, 0.7]),
    "bitc_k211_g8_nb2": lambda: T.tiny_fcc(kmesh=(2, 1, 1), grid=8, ecut=2.0, nb=2, a=6.0, occ=[1.0, 0.7],
                                           left_mix=0.15),
}


@pytest.mark.parametrize("name", list(CASES))
def test_small_fcc_fixed_point_vs_oracle(name):
    w = CASES[name]()
    bitc = w.left is not None
    _say(f"[gpu] scf {name}: run to convergence, then the oracle checks the fixed point")
    op = tc.from_workload(w, precision=tc.TC_PREC_FP64)
    hist, n = op.scf(max_iter=1500, pmax=2, etol=1e-13, otol=1e-9)
    E = op.energy()[0]
    wr, wl, we, R, L = _fixed_point(w, op, bitc)
    op.close()
    Eo = S.energy(w, R, L)
    _say(f"    {n} iterations, E = {E!r} (oracle at these orbitals {Eo!r}); invariance residual right "
         f"{wr:.2e} left {wl:.2e}; eigenvalue gap to the lowest {we:.2e}")
    assert n < 1500
    assert abs(E - Eo) < 1e-10 * abs(Eo)
    assert wr < 1e-6 and wl < 1e-6
    assert we < 1e-6


def test_fp32_and_mixing_reach_the_same_fixed_point():
    w = CASES["tc_k211_g8_nb1"]()
    res = {}
    for name, prec, mix in (("fp64", tc.TC_PREC_FP64, 1.0), ("fp32", tc.TC_PREC_FP32, 1.0),
                            ("fp64_mix", tc.TC_PREC_FP64, 0.5)):
        op = tc.from_workload(w, precision=prec)
        _, n = op.scf(max_iter=1500, pmax=2, etol=1e-13, mix=mix, otol=1e-9)
        res[name] = op.energy()[0]
        assert op.get_orbitals(0).shape == w.right[0].shape     # the loop's orbitals alone at the end
        op.close()
    _say(f"[gpu] scf fixed point: {res}")
    assert abs(res["fp32"] - res["fp64"]) < 1e-6 * abs(res["fp64"])
    assert abs(res["fp64_mix"] - res["fp64"]) < 1e-7 * abs(res["fp64"])


def test_errors():
    w = CASES["tc_k211_g8_nb1"]()
    op = tc.from_workload(w, precision=tc.TC_PREC_FP64)
    for bad in (dict(max_iter=0), dict(pmax=-1), dict(pmax=17), dict(etol=0.0), dict(mix=0.0), dict(mix=1.5)):
        with pytest.raises(tc.TCError, match="status -1"):
            op.scf(**bad)
    op.close()
