"""Physics invariants of the oracle: supercell folding, orbital mixing, Hermiticity, energy identities."""
import math

import numpy as np
import pytest
import torch

import tcinputs as T
from oracle.fftroute import ALL_TERMS, MULT, Problem, TERMS2, TERMS3


def _fold_to_supercell(w):
    """Gamma-only description of the same orbitals on the cell doubled along a1 (k-mesh n1 x 1 x 1)."""
    n1 = w.kmesh[0]
    assert w.kmesh[1] == w.kmesh[2] == 1
    lat = np.array(w.lattice)
    lat[0] *= n1
    mill, coef, occ = [], [], []
    allm = []
    for ik in range(n1):
        allm.append(w.miller[ik] * np.array([n1, 1, 1]) + np.array([ik, 0, 0]))
    M = np.unique(np.concatenate(allm), axis=0)
    rows = []
    for ik in range(n1):
        idx = [np.where(np.all(M == m[None], 1))[0][0] for m in allm[ik]]
        for b in range(w.right[ik].shape[0]):
            c = np.zeros(M.shape[0], dtype=np.complex128)
            c[idx] = w.right[ik][b]
            rows.append(c)
            occ.append(w.occ[ik][b])
    grid = (w.grid[0] * n1, w.grid[1], w.grid[2])
    return w.replace(lattice=lat, kmesh=(1, 1, 1), grid=grid, miller=[M.astype(np.int32)],
                     right=[np.array(rows)], occ=[np.array(occ)])


def test_supercell_folding_including_corrections():
    w = T.tiny_fcc(kmesh=(2, 1, 1), grid=12, ecut=2.0, nb=2, a=6.0, occ=[1.0, 0.8])
    ws = _fold_to_supercell(w)
    Ep, pp = Problem(w).energy(per_term=True)
    Es, ps = Problem(ws).energy(per_term=True)
    for k in pp:
        assert float(ps[k]) / 2 == pytest.approx(float(pp[k]), rel=1e-10, abs=1e-13), k
    assert float(Es) / 2 == pytest.approx(float(Ep), rel=1e-11)


def _rand_unitary(n, rng):
    z = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    q, r = np.linalg.qr(z)
    return q * (np.diag(r) / np.abs(np.diag(r)))[None, :]


def test_unitary_mixing_invariance_tc():
    w = T.tiny_fcc(kmesh=(2, 1, 1), grid=8, ecut=2.0, nb=3, a=6.0)
    rng = np.random.default_rng(5)
    U = [_rand_unitary(3, rng) for _ in w.right]
    w2 = w.replace(right=[u @ c for u, c in zip(U, w.right)])
    p1, p2 = Problem(w), Problem(w2)
    assert float(p2.energy()) == pytest.approx(float(p1.energy()), rel=1e-12)
    g1 = sum(p1.operator(s=0))
    g2 = sum(p2.operator(s=0))
    for ik, u in enumerate(U):
        J = p1.sel(0, ik)
        mixed = torch.einsum("ab,b...->a...", torch.as_tensor(u), g1[J])
        assert torch.max(torch.abs(mixed - g2[J])) < 1e-11 * torch.max(torch.abs(g1))


def test_biorthogonal_gl_invariance_and_biorthonormality():
    w = T.tiny_fcc(kmesh=(2, 1, 1), grid=8, ecut=2.0, nb=2, a=6.0, left_mix=0.2, seed_offset=11)
    rng = np.random.default_rng(9)
    M = [rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2)) + 2 * np.eye(2) for _ in w.right]
    N = [rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2)) + 2 * np.eye(2) for _ in w.right]
    w2 = w.replace(right=[m @ c for m, c in zip(M, w.right)], left=[n @ c for n, c in zip(N, w.left)])
    p1, p2 = Problem(w), Problem(w2)
    for cr, cl in zip(p2.cr, p2.cl):
        S = torch.conj(cl) @ cr.T
        assert torch.max(torch.abs(S - torch.eye(2))) < 1e-13
    assert float(p2.energy()) == pytest.approx(float(p1.energy()), rel=1e-11)


def _matrix(pr, terms, ik):
    g2, g3 = pr.operator(terms=terms, s=0)
    g = g2 + g3
    J = pr.sel(0, ik)
    phi = pr.orb[0]["phi"][J]
    return pr.omega * torch.einsum("a...,b...->ab", torch.conj(phi), g[J]) / pr.nr


@pytest.mark.parametrize("part", ["fock_u0", "v2a", "three_body"])
def test_hermiticity_tc(part):
    # two occupied + one empty band per k so the check reaches outside the occupied space
    w = T.tiny_fcc(kmesh=(2, 1, 1), grid=8, ecut=2.0, nb=3, a=6.0, occ=[1.0, 1.0, 0.0])
    if part == "fock_u0":
        pr, terms = Problem(w.replace(A=(0.0, 0.0))), TERMS2
    elif part == "v2a":
        pr, terms = Problem(w), ("2ah", "2ax")
    else:
        pr, terms = Problem(w), TERMS3
    for ik in range(2):
        M = _matrix(pr, terms, ik)
        assert torch.max(torch.abs(M - M.conj().T)) < 1e-12 * torch.max(torch.abs(M)), part


def test_gradient_term_energy_identities():
    """<2bx2> = <2bx1> and <2bh2> = <2bh1> (transposition of the discrete convolutions)."""
    w = T.tiny_fcc(kmesh=(2, 1, 1), grid=8, ecut=2.0, nb=2, a=6.0, left_mix=0.1, seed_offset=3, occ=[1.0, 0.5])
    _, p = Problem(w).energy(per_term=True)
    assert float(p["2bx2"]) == pytest.approx(float(p["2bx1"]), rel=1e-11)
    assert float(p["2bh2"]) == pytest.approx(float(p["2bh1"]), rel=1e-11)


def test_energy_is_quadratic_in_A():
    """At fixed C every kernel is linear (u~, lap u~) or quadratic ((grad u)^2~, three-body) in A."""
    w = T.tiny_fcc(kmesh=(2, 1, 1), grid=8, ecut=2.0, nb=2, a=6.0)
    C = w.C
    grid = [(a1, a2) for a1 in (0.5, 1.0, 1.7) for a2 in (0.4, 1.1, 1.6)]
    E = np.array([float(Problem(w.replace(A=a, C=C)).energy()) for a in grid])
    X = np.array([[1, a1, a2, a1 * a1, a1 * a2, a2 * a2] for a1, a2 in grid])
    coef, res, *_ = np.linalg.lstsq(X, E, rcond=None)
    assert np.max(np.abs(X @ coef - E)) < 1e-12 * np.max(np.abs(E))


def test_target_sample_rows_equal_full_rows():
    """Restricting the oracle to a sample of targets leaves those rows unchanged (full-size sampled checks)."""
    w = T.tiny_fcc(kmesh=(2, 2, 1), grid=8, ecut=2.0, nb=2, a=6.0, occ=[1.0, 0.6])
    full, part = Problem(w), Problem(w)
    part.restrict_targets([1, 6])
    for t in ("2ax", "2bx1", "2bx2", "3a3", "3a4", "3b3", "3b4", "3b5", "3b6", "2ah", "3a1"):
        a, b = full.term(t, 0), part.term(t, 0)
        for j in (1, 6):
            assert torch.max(torch.abs(b[j] - a[j])) <= 1e-14 * torch.max(torch.abs(a)), (t, j)


@pytest.mark.parametrize("left_mix", [None, 0.15])
def test_coefficient_output_obeys_parseval(left_mix):
    """Pins to_coeff against the real-space bracket: for every orbital, <chi_p|g_p> over the cell (grid
    sum, Sec. 2.2's periodic transform not involved) equals sum_G conj(c~_p(G)) (Hc)_p(G) on its plane-wave
    set, with c~ the left coefficients (the right ones in TC mode).  A wrong sqrt(Omega) or 1/N_r in the
    coefficient output, or a misplaced gather, breaks it."""
    w = T.tiny_fcc(kmesh=(2, 1, 1), grid=8, ecut=2.0, nb=2, a=6.0, occ=[1.0, 0.7], left_mix=left_mix)
    pr = Problem(w)
    g = sum(MULT.get(t, 1) * pr.term(t, 0) for t in ALL_TERMS)
    hc = pr.to_coeff(g)
    bra = pr.braket(0, g)
    cl = pr.cr if pr.cl is None else pr.cl
    for ik in range(pr.nk):
        J = pr.sel(0, ik)
        lhs = torch.sum(torch.conj(cl[ik]) * hc[ik], 1)
        assert torch.max(torch.abs(lhs - bra[J])) <= 1e-13 * torch.max(torch.abs(bra))
    assert float(torch.max(torch.abs(bra))) > 1e-3
