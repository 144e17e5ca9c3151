"""Spin-polarised TC mode of the HIP path through the C ABI: each spin channel has its own orbitals.

Against the FP64 oracle on the same inputs: every term of both spin channels, the totals, the energy
and its parts, the orbital energies of both channels (FP64 and FP32), the gradient of each channel's
coefficients and of A, C (autograd), each channel's operator on trial vectors, and the fixed point of
the two-channel SCF loop (per-channel plane-wave matrices); in the biorthogonal mode (a left set per
channel) every term, the energy, the orbital energies, the right and left gradients and the trial
vectors.  Independent of the oracle: two identical channels reproduce the unpolarised run and its SCF
iterates (TC and biorthogonal), and exchanging the channels exchanges the outputs and keeps the energy.
Left orbitals in one channel only fail with TC_ERR_STATE.
"""
import numpy as np
import pytest

import tcinputs as T
from oracle.fftroute import ALL_TERMS, MULT, Problem

pytestmark = pytest.mark.gpu

tc = pytest.importorskip("paper_2302_07420_amd")

FP64_TOL = 1e-10
FP32_TOL = 2e-6


def _say(msg):
    print(msg, flush=True)


def relerr(a, b):
    scale = max(np.abs(x).max() for x in b)
    return max(np.abs(x - y).max() for x, y in zip(a, b)) / scale


CASES = {
    "fcc_k211_g8_pol": lambda: T.polarized(T.tiny_fcc(kmesh=(2, 1, 1), grid=8, ecut=2.0, nb=2, a=6.0,
                                                      occ=[1.0, 0.7]), 31, occ_dn=[0.9, 0.2]),
    "fcc_k221_g12_pol_empty_band": lambda: T.polarized(T.tiny_fcc(kmesh=(2, 2, 1), grid=12, ecut=2.0, nb=3, a=6.0,
                                                                  occ=[1.0, 0.8, 0.3], seed_offset=5), 33,
                                                       occ_dn=[1.0, 0.0, 0.0]),
    "fcc_k121_g16_pol": lambda: T.polarized(T.tiny_fcc(kmesh=(1, 2, 1), grid=16, ecut=3.0, nb=2, a=7.0,
                                                       seed_offset=9), 34, mix=0.5),
    # biorthogonal mode: a left set per channel
    "fcc_k211_g8_bitc_pol": lambda: T.polarized(T.tiny_fcc(kmesh=(2, 1, 1), grid=8, ecut=2.0, nb=2, a=6.0,
                                                           occ=[1.0, 0.7], left_mix=0.15, seed_offset=7), 35,
                                                occ_dn=[0.9, 0.2]),
    "fcc_k221_g12_bitc_pol_empty_band": lambda: T.polarized(T.tiny_fcc(kmesh=(2, 2, 1), grid=12, ecut=2.0, nb=3,
                                                                       a=6.0, occ=[1.0, 0.8, 0.3], left_mix=0.1,
                                                                       seed_offset=5), 37, occ_dn=[1.0, 0.0, 0.0]),
    "fcc_k121_g16_bitc_pol": lambda: T.polarized(T.tiny_fcc(kmesh=(1, 2, 1), grid=16, ecut=3.0, nb=2, a=7.0,
                                                            left_mix=0.2, seed_offset=9), 36, mix=0.5),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    w = CASES[request.param]()
    pr = Problem(w)
    assert pr.polarized
    per = {s: {t: [c.numpy() for c in pr.to_coeff(MULT.get(t, 1) * pr.term(t, s), s)] for t in ALL_TERMS}
           for s in (0, 1)}
    tot = {s: [sum(per[s][t][k] for t in ALL_TERMS) for k in range(w.nk)] for s in (0, 1)}
    E, parts = pr.energy(per_term=True)
    eps = np.stack([(pr.kinetic(s) + pr.braket(s, sum(MULT.get(t, 1) * pr.term(t, s) for t in ALL_TERMS)))
                    .numpy().reshape(w.nk, -1) for s in (0, 1)])
    return request.param, w, per, tot, float(E), {k: float(v) for k, v in parts.items()}, eps


def test_every_term_fp64(case):
    name, w, per, tot, *_ = case
    for t in ALL_TERMS:
        _say(f"[gpu] polarised {name} fp64 term {t}")
        op = tc.from_workload(w, precision=tc.TC_PREC_FP64, terms=tc.TERM_BITS[t] | tc.TERM_BITS["corr"])
        got = op.apply()
        op.close()
        for s in (0, 1):
            scale = max(np.abs(x).max() for x in tot[s])
            err = max(np.abs(g - r).max() for g, r in zip(got[s], per[s][t])) / scale
            assert err < FP64_TOL, (t, s, err)


@pytest.mark.parametrize("prec,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
def test_total_energy_and_orbital_energies(case, prec, tol):
    name, w, per, tot, E, parts, eps = case
    _say(f"[gpu] polarised {name} {prec} total")
    op = tc.from_workload(w, precision=tc.TC_PREC_FP64 if prec == "fp64" else tc.TC_PREC_FP32)
    got = op.apply()
    Eg, pg = op.energy()
    eg = op.orbital_energies()
    op.close()
    for s in (0, 1):
        err = relerr(got[s], tot[s])
        _say(f"    spin {s}: max |H c - oracle| / max = {err:.3e}")
        assert err < tol, (s, err)
    assert abs(Eg - E) < tol * abs(E), (Eg, E)
    assert abs(pg["kinetic"] - parts["T"]) < tol * abs(E)
    e2 = sum(parts[t] for t in ALL_TERMS if t.startswith("2"))
    e3 = sum(parts[t] for t in ALL_TERMS if t.startswith("3"))
    assert abs(pg["two_body"] - e2) < tol * abs(E), (pg["two_body"], e2)
    assert abs(pg["three_body"] - e3) < tol * abs(E), (pg["three_body"], e3)
    assert eg.shape == eps.shape
    erre = np.abs(eg - eps).max() / np.abs(eps).max()
    _say(f"    orbital energies: {erre:.3e}")
    assert erre < tol


def test_identical_channels_reproduce_unpolarized():
    """Both channels loaded with the same orbitals and fillings: the unpolarised run's outputs."""
    w = T.tiny_fcc(kmesh=(2, 2, 1), grid=12, ecut=2.0, nb=3, a=6.0, occ=[1.0, 0.9, 0.0])
    _say("[gpu] polarised identical channels fcc_k221_g12")
    op = tc.from_workload(w, precision=tc.TC_PREC_FP64)
    ref = op.apply()
    E0, p0 = op.energy()
    e0 = op.orbital_energies()
    op.close()
    wp = w.replace(right_dn=list(w.right), occ_dn=list(w.occ))
    op = tc.from_workload(wp, precision=tc.TC_PREC_FP64)
    got = op.apply()
    E1, p1 = op.energy()
    e1 = op.orbital_energies()
    op.close()
    for s in (0, 1):
        assert relerr(got[s], ref) < 1e-12
        assert np.abs(e1[s] - e0).max() < 1e-12 * np.abs(e0).max()
    assert abs(E1 - E0) < 1e-12 * abs(E0)


def test_exchanging_channels_exchanges_outputs():
    w = T.polarized(T.tiny_fcc(kmesh=(2, 1, 1), grid=8, ecut=2.0, nb=2, a=6.0, occ=[1.0, 0.7]), 9,
                    occ_dn=[0.8, 0.1])
    ws = w.replace(right=w.right_dn, right_dn=w.right, occ=w.occ_dn, occ_dn=w.occ)
    _say("[gpu] polarised channel exchange fcc_k211_g8")
    outs, Es = [], []
    for x in (w, ws):
        op = tc.from_workload(x, precision=tc.TC_PREC_FP64)
        outs.append(op.apply())
        Es.append(op.energy()[0])
        op.close()
    assert abs(Es[1] - Es[0]) < 1e-12 * abs(Es[0])
    for s in (0, 1):
        assert relerr(outs[1][1 - s], outs[0][s]) < 1e-12


def test_left_orbitals_in_one_channel_only_are_rejected():
    w = T.polarized(T.tiny_fcc(kmesh=(2, 1, 1), grid=8, ecut=2.0, nb=2, a=6.0, occ=[1.0, 0.7]), 9)
    _say("[gpu] polarised: left orbitals in the down channel only")
    op = tc.from_workload(w, precision=tc.TC_PREC_FP64)
    op.load_orbitals(0, w.right_dn[0], w.occ_dn[0], left=w.right_dn[0], spin=1)
    with pytest.raises(tc.TCError, match="status"):
        op.apply()
    op.close()
    # a missing down channel is reported before any work
    op = tc.TCOperator()
    op.set_cell(w.lattice)
    op.set_kmesh(*w.kmesh)
    op.set_grid(*w.grid)
    for ik, m in enumerate(w.miller):
        op.set_basis(ik, m)
    op.set_jastrow(w.A, w.C)
    op.set_options(tc.TC_PREC_FP64, w.alpha, True, tc.TERM_ALL)
    op.set_nspin(2)
    for ik in range(w.nk):
        op.load_orbitals(ik, w.right[ik], w.occ[ik])
    with pytest.raises(tc.TCError, match="status"):
        op.apply()
    op.close()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_polarized_gradient_vs_oracle(prec):
    """2 dE/dc* of each spin channel's own coefficients and dE/dA, dE/dC against the oracle's autograd
    (one application with the gradient tables, both channels, scale 2 per channel)."""
    from oracle import grad as OG

    w = T.polarized(T.tiny_fcc(kmesh=(2, 1, 1), grid=8, ecut=2.0, nb=2, a=6.0, occ=[1.0, 0.6]), 41,
                    occ_dn=[0.9, 0.3])
    E, gu, gd, gA, gC = OG.energy_and_grad_polarized(w)
    _say(f"[gpu] polarized backward {prec} vs oracle autograd")
    op = tc.from_workload(w, precision=tc.TC_PREC_FP64 if prec == "fp64" else tc.TC_PREC_FP32)
    Eg, _ = op.energy()
    (hu, hd), dA, dC = op.backward()
    op.close()
    tol = 1e-10 if prec == "fp64" else 2e-6
    scale = max(np.abs(x).max() for x in gu + gd)
    err = max(np.abs(a - b).max() for a, b in zip(hu + hd, gu + gd)) / scale
    perr = max(np.abs(dA - gA).max(), np.abs(dC - gC).max()) / max(np.abs(gA).max(), np.abs(gC).max())
    _say(f"    E {Eg!r} vs {E!r}; grad rel err {err:.3e}; params rel err {perr:.3e}")
    assert abs(Eg - E) < (1e-10 if prec == "fp64" else 1e-6) * abs(E)
    assert err < tol
    assert perr < (1e-10 if prec == "fp64" else 1e-6)


def _pol_small():
    return T.polarized(T.tiny_fcc(kmesh=(2, 1, 1), grid=8, ecut=2.0, nb=2, a=6.0, occ=[1.0, 0.6]), 41,
                       occ_dn=[0.9, 0.3])


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 2e-6)])
def test_polarized_trial_vectors_vs_oracle(prec, tol):
    """tc_apply with two channels: each channel's trial vectors against its own operator.  The oracle adds
    them to their channel as bands of zero filling (targets of every term, partners of none)."""
    w = _pol_small()
    rng = np.random.default_rng(5)
    nv = 3
    B = 2 * np.pi * np.linalg.inv(np.asarray(w.lattice)).T
    env = [np.exp(-0.15 * np.sum(((w.kfrac[k][None, :] + m) @ B) ** 2, 1)) for k, m in enumerate(w.miller)]
    vecs = [[(rng.standard_normal((nv, m.shape[0])) + 1j * rng.standard_normal((nv, m.shape[0]))) * e
             for m, e in zip(w.miller, env)] for _ in range(2)]
    od = w.occ_dn
    wx = w.replace(right=[np.concatenate([a, v]) for a, v in zip(w.right, vecs[0])],
                   right_dn=[np.concatenate([a, v]) for a, v in zip(w.right_dn, vecs[1])],
                   occ=[np.concatenate([o, np.zeros(nv)]) for o in w.occ],
                   occ_dn=[np.concatenate([o, np.zeros(nv)]) for o in od])
    pr = Problem(wx)
    nb = w.right[0].shape[0]
    ref = []
    for s in (0, 1):
        g = sum(MULT.get(t, 1) * pr.term(t, s) for t in ALL_TERMS)
        ref.append([c.numpy()[nb:] for c in pr.to_coeff(g, s)])
    _say(f"[gpu] polarized trial vectors {prec} vs oracle")
    op = tc.from_workload(w, precision=tc.TC_PREC_FP64 if prec == "fp64" else tc.TC_PREC_FP32)
    op.energy()
    got = op.apply_vectors(vecs)
    op.close()
    scale = max(np.abs(x).max() for r in ref for x in r)
    err = max(np.abs(a - b).max() for s in (0, 1) for a, b in zip(got[s], ref[s])) / scale
    _say(f"    max element error / max |h v| = {err:.3e}")
    assert err < tol


def test_polarized_scf_with_equal_channels_follows_the_unpolarized_loop():
    """Two identical channels are the unpolarised problem: the two-channel block-Davidson loop (one
    subspace per channel and k-point) takes the same steps and energies."""
    w = T.tiny_fcc(kmesh=(2, 1, 1), grid=8, ecut=2.0, nb=2, a=6.0, occ=[1.0, 0.7])
    wp = w.replace(right_dn=[c.copy() for c in w.right], occ_dn=[o.copy() for o in w.occ])
    _say("[gpu] polarized scf with equal channels vs the unpolarized loop")
    out = []
    for ww in (w, wp):
        op = tc.from_workload(ww, precision=tc.TC_PREC_FP64)
        hist, n = op.scf(max_iter=5, pmax=2, etol=1e-300, otol=0.0)
        out.append(np.array(hist[:n]))
        op.close()
    _say(f"    energies {out[0]} vs {out[1]}")
    assert len(out[0]) == len(out[1])
    np.testing.assert_allclose(out[1], out[0], rtol=1e-10)


def test_polarized_scf_fixed_point_vs_oracle():
    """A spin-polarised loop to convergence; the oracle then builds each channel's matrix of T + h from the
    final orbitals of both channels: each channel's orbitals span an invariant subspace of its matrix,
    with its lowest eigenvalues."""
    from oracle import scf as S

    w = _pol_small()
    _say("[gpu] polarized scf to convergence; fixed point checked by the oracle per channel")
    op = tc.from_workload(w, precision=tc.TC_PREC_FP64)
    hist, n = op.scf(max_iter=1500, pmax=2, etol=1e-13, otol=1e-9)
    E = op.energy()[0]
    R = [[op.get_orbitals(k, spin=s) for k in range(w.nk)] for s in (0, 1)]
    op.close()
    worst_r = worst_e = 0.0
    for s in (0, 1):
        H = S.operator_matrices(w, R[0], spin=s, right_dn=R[1])
        for k in range(w.nk):
            Phi = R[s][k].T
            Hk = H[k]
            Ek = Phi.conj().T @ Hk @ Phi
            assert np.abs(Phi.conj().T @ Phi - np.eye(Phi.shape[1])).max() < 1e-10
            worst_r = max(worst_r, np.abs(Hk @ Phi - Phi @ Ek).max() / np.abs(Hk).max())
            lam = np.sort(np.linalg.eigvals(Hk).real)
            mine = np.sort(np.linalg.eigvals(Ek).real)
            worst_e = max(worst_e, np.abs(mine - lam[: len(mine)]).max())
    from oracle import grad as OG
    Eo = OG.energy_polarized(w, up=R[0], dn=R[1])
    _say(f"    {n} iterations, E = {E!r} (oracle {Eo!r}); invariance residual {worst_r:.2e}; "
         f"eigenvalue gap {worst_e:.2e}")
    assert n < 1500
    assert abs(E - Eo) < 1e-10 * abs(Eo)
    assert worst_r < 1e-6
    assert worst_e < 1e-6


def _bitc_pol():
    return CASES["fcc_k211_g8_bitc_pol"]()


def test_bitc_identical_channels_reproduce_unpolarized_bitc():
    """Two biorthogonal channels with the same pair and fillings: the unpolarised biorthogonal run."""
    w = T.tiny_fcc(kmesh=(2, 2, 1), grid=12, ecut=2.0, nb=3, a=6.0, occ=[1.0, 0.9, 0.0], left_mix=0.1,
                   seed_offset=5)
    _say("[gpu] polarised biorthogonal, identical channels fcc_k221_g12")
    op = tc.from_workload(w, precision=tc.TC_PREC_FP64)
    ref = op.apply()
    E0, _ = op.energy()
    e0 = op.orbital_energies()
    op.close()
    wp = w.replace(right_dn=list(w.right), left_dn=list(w.left), occ_dn=list(w.occ))
    op = tc.from_workload(wp, precision=tc.TC_PREC_FP64)
    got = op.apply()
    E1, _ = op.energy()
    e1 = op.orbital_energies()
    op.close()
    for s in (0, 1):
        assert relerr(got[s], ref) < 1e-12
        assert np.abs(e1[s] - e0).max() < 1e-12 * np.abs(e0).max()
    assert abs(E1 - E0) < 1e-12 * abs(E0)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 2e-6)])
def test_bitc_polarized_gradients_vs_oracle(prec, tol):
    """The right and left gradients of each channel (its own pair) and dA, dC against the oracle's
    autograd at the biorthonormalised pairs."""
    from oracle import grad as OG

    w = _bitc_pol()
    pairs = OG.bitc_pair_polarized(w)
    E, gru, glu, grd, gld, gA, gC = OG.energy_and_grad_bitc_polarized(w, *pairs)
    _say(f"[gpu] polarised biorthogonal backward {prec} vs oracle autograd")
    op = tc.from_workload(w, precision=tc.TC_PREC_FP64 if prec == "fp64" else tc.TC_PREC_FP32)
    Eg, _ = op.energy()
    gr, gl, dA, dC = op.backward_lr()
    op.close()
    assert abs(Eg - E) < tol * abs(E)
    for got, ref in ((gr[0], gru), (gr[1], grd), (gl[0], glu), (gl[1], gld)):
        err = relerr(got, ref)
        _say(f"    gradient error {err:.3e}")
        assert err < tol
    scale = max(np.abs(gA).max(), np.abs(gC).max())
    assert np.abs(dA - gA).max() < tol * scale and np.abs(dC - gC).max() < tol * scale


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 2e-6)])
def test_bitc_polarized_trial_vectors_vs_oracle(prec, tol):
    """tc_apply in the biorthogonal mode with two channels: the oracle takes each channel's
    biorthonormalised pair and adds the vectors to that channel as bands of zero filling (right and left)."""
    from oracle import grad as OG

    w = _bitc_pol()
    ru, lu, rd, ld = OG.bitc_pair_polarized(w)
    rng = np.random.default_rng(7)
    nv = 2
    B = 2 * np.pi * np.linalg.inv(np.asarray(w.lattice)).T
    env = [np.exp(-0.15 * np.sum(((w.kfrac[k][None, :] + m) @ B) ** 2, 1)) for k, m in enumerate(w.miller)]
    vecs = [[(rng.standard_normal((nv, m.shape[0])) + 1j * rng.standard_normal((nv, m.shape[0]))) * e
             for m, e in zip(w.miller, env)] for _ in range(2)]
    cat = lambda a, v: [np.concatenate([x, y]) for x, y in zip(a, v)]
    wx = w.replace(right=cat(ru, vecs[0]), left=cat(lu, vecs[0]), right_dn=cat(rd, vecs[1]),
                   left_dn=cat(ld, vecs[1]), occ=[np.concatenate([o, np.zeros(nv)]) for o in w.occ],
                   occ_dn=[np.concatenate([o, np.zeros(nv)]) for o in w.occ_dn])
    pr = Problem(wx, biorthogonalize=False)
    nb = w.right[0].shape[0]
    ref = []
    for s in (0, 1):
        g = sum(MULT.get(t, 1) * pr.term(t, s) for t in ALL_TERMS)
        ref.append([c.numpy()[nb:] for c in pr.to_coeff(g, s)])
    _say(f"[gpu] polarised biorthogonal trial vectors {prec} vs oracle")
    op = tc.from_workload(w, precision=tc.TC_PREC_FP64 if prec == "fp64" else tc.TC_PREC_FP32)
    op.energy()
    got = op.apply_vectors(vecs)
    op.close()
    scale = max(np.abs(x).max() for r in ref for x in r)
    err = max(np.abs(a - b).max() for s in (0, 1) for a, b in zip(got[s], ref[s])) / scale
    _say(f"    max element error / max |h v| = {err:.3e}")
    assert err < tol


def test_bitc_polarized_scf_with_equal_channels_follows_the_unpolarized_loop():
    """Two identical biorthogonal channels: the two-channel BITC-SCF loop takes the unpolarised loop's
    steps and energies."""
    w = T.tiny_fcc(kmesh=(2, 1, 1), grid=8, ecut=2.0, nb=2, a=6.0, occ=[1.0, 0.7], left_mix=0.15, seed_offset=7)
    wp = w.replace(right_dn=[c.copy() for c in w.right], left_dn=[c.copy() for c in w.left],
                   occ_dn=[o.copy() for o in w.occ])
    _say("[gpu] polarised biorthogonal scf with equal channels vs the unpolarised loop")
    out = []
    for ww in (w, wp):
        op = tc.from_workload(ww, precision=tc.TC_PREC_FP64)
        hist, n = op.scf(max_iter=5, pmax=2, etol=1e-300, otol=0.0)
        out.append(np.array(hist[:n]))
        op.close()
    _say(f"    energies {out[0]} vs {out[1]}")
    assert len(out[0]) == len(out[1])
    np.testing.assert_allclose(out[1], out[0], rtol=1e-10)


@pytest.mark.parametrize("name", ["fcc_k221_g12_pol_empty_band", "fcc_k211_g8_bitc_pol"])
def test_polarized_pair_store_on_and_off_agree(name):
    """Two channels with the resident store of pass-A z-stage outputs (one region per channel, read by the
    occupied pass and pass A), with a budget that leaves it half of the partner columns (TC mode: the
    triangular store of P/2 columns per channel; the biorthogonal mode then keeps none), and without it
    (each pass forms its own pairs): the same operator."""
    w = CASES[name]()
    P, NR = w.nk * w.nband, int(np.prod(w.grid))
    bitc = w.left is not None
    keep = P * ((8 if bitc else 5) + 4) * NR * 16 * min(8, P)
    q1 = P // 2
    tri = q1 * (q1 + 1) // 2 + (P - q1) * q1
    half = keep + 5 * 2 * NR * 16 * (P * q1 if bitc else tri)
    _say(f"[gpu] polarised {name}: pair store on / half / off")
    res = []
    for kw in (dict(), dict(mem_budget=half), dict(pair_store=False)):
        op = tc.from_workload(w, precision=tc.TC_PREC_FP64, **kw)
        res.append((op.apply(), op.energy()[0], op.orbital_energies()))
        op.close()
    for r in res[1:]:
        for s in (0, 1):
            assert relerr(r[0][s], res[0][0][s]) < 1e-12
        assert abs(r[1] - res[0][1]) < 1e-12 * abs(res[0][1])
        assert np.abs(r[2] - res[0][2]).max() < 1e-12 * np.abs(res[0][2]).max()
