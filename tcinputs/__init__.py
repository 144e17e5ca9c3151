"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module holds geometry and random-number plumbing only: lattice vectors,
Gamma-centred Monkhorst-Pack k lists, plane-wave index sets inside a kinetic
cutoff, random orbital coefficients and occupations.  It contains none of the
transcorrelated method's arithmetic (no kernels, no transforms, no terms), so
that both the CPU oracle and the HIP library can consume the same inputs
without sharing any of the computation they are compared on.

Conventions (also used by the C ABI):
  * lattice rows are a1, a2, a3 in bohr; reciprocal rows b_j satisfy
    a_i . b_j = 2 pi delta_ij;
  * k-points are Gamma-centred: k = (i1/n1, i2/n2, i3/n3) in units of b, with
    flat index ik = (i1*n2 + i2)*n3 + i3 (fractions kept in [0, 1));
  * an orbital's coefficients c(G) over Miller indices m give the cell-periodic
    part phi(r) = Omega^{-1/2} sum_G c(G) exp(i G.r), sum |c|^2 = 1.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np

SEED_BASE = 230207420


def sc_lattice(L: float) -> np.ndarray:
    return np.eye(3) * float(L)


def fcc_lattice(a: float) -> np.ndarray:
    h = 0.5 * float(a)
    return np.array([[0.0, h, h], [h, 0.0, h], [h, h, 0.0]])


def reciprocal(lattice: np.ndarray) -> np.ndarray:
    return 2.0 * math.pi * np.linalg.inv(np.asarray(lattice, dtype=np.float64)).T


def kmesh_fractions(n1: int, n2: int, n3: int, shift=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Fractional k-points (i + s) / n of an n1 x n2 x n3 Monkhorst-Pack mesh, shift s in mesh units
    (0: Gamma-centred)."""
    s1, s2, s3 = (float(x) for x in shift)
    out = []
    for i1 in range(n1):
        for i2 in range(n2):
            for i3 in range(n3):
                out.append(((i1 + s1) / n1, (i2 + s2) / n2, (i3 + s3) / n3))
    return np.array(out, dtype=np.float64)


def miller_sphere(lattice: np.ndarray, kfrac, ecut: float) -> np.ndarray:
    """Miller indices m with |k+G|^2/2 <= ecut, sorted by (|k+G|^2, m)."""
    B = reciprocal(lattice)
    kc = math.sqrt(2.0 * ecut)
    bmin = min(np.linalg.norm(B, axis=1))
    # bound on |m_i| from the dual basis
    mmax = int(math.ceil(kc * np.max(np.linalg.norm(np.asarray(lattice), axis=1)) / (2 * math.pi))) + 2
    r = np.arange(-mmax, mmax + 1)
    M = np.stack(np.meshgrid(r, r, r, indexing="ij"), -1).reshape(-1, 3)
    kg = (M + np.asarray(kfrac)[None, :]) @ B
    e = 0.5 * np.sum(kg * kg, axis=1)
    keep = e <= ecut + 1e-12
    M, e = M[keep], e[keep]
    order = np.lexsort((M[:, 2], M[:, 1], M[:, 0], np.round(e, 12)))
    del bmin
    return M[order].astype(np.int32)


def miller_norm2(mmax2: int) -> np.ndarray:
    """All integer vectors with |m|^2 <= mmax2 (simple cubic shells)."""
    r = int(math.isqrt(mmax2)) + 1
    rr = np.arange(-r, r + 1)
    M = np.stack(np.meshgrid(rr, rr, rr, indexing="ij"), -1).reshape(-1, 3)
    n2 = np.sum(M * M, axis=1)
    M = M[n2 <= mmax2]
    n2 = n2[n2 <= mmax2]
    order = np.lexsort((M[:, 2], M[:, 1], M[:, 0], n2))
    return M[order].astype(np.int32)


@dataclasses.dataclass
class Workload:
    """One unpolarized synthetic problem (both spin channels identical)."""
    name: str
    lattice: np.ndarray            # (3,3) rows a_i
    kmesh: tuple                   # (n1,n2,n3), Gamma-centred
    grid: tuple                    # (N1,N2,N3)
    miller: List[np.ndarray]       # per k: (npw,3) int32
    right: List[np.ndarray]        # per k: (nb,npw) complex128
    left: Optional[List[np.ndarray]]  # per k or None (TC mode)
    occ: List[np.ndarray]          # per k: (nb,) fillings per spin-orbital
    A: tuple                       # (A_par, A_anti)
    C: tuple                       # (C_par, C_anti)
    alpha: float                   # Gygi-Baldereschi auxiliary exponent
    nelec_cell: int
    # spin-polarised input: the down-spin channel's own orbitals and fillings (None: same as up)
    right_dn: Optional[List[np.ndarray]] = None
    left_dn: Optional[List[np.ndarray]] = None
    occ_dn: Optional[List[np.ndarray]] = None
    # band (zero-weight) k-points off the mesh: fractional k, plane waves, orbitals and fillings
    band_k: Optional[np.ndarray] = None
    band_miller: Optional[List[np.ndarray]] = None
    band_right: Optional[List[np.ndarray]] = None
    band_occ: Optional[List[np.ndarray]] = None
    # shift of the k-mesh in mesh units (0: Gamma-centred; 1/2: the Monkhorst-Pack shift of an even mesh)
    kshift: tuple = (0.0, 0.0, 0.0)

    @property
    def omega(self) -> float:
        return abs(float(np.linalg.det(self.lattice)))

    @property
    def nk(self) -> int:
        return int(np.prod(self.kmesh))

    @property
    def kfrac(self) -> np.ndarray:
        return kmesh_fractions(*self.kmesh, shift=self.kshift)

    @property
    def nband(self) -> int:
        return int(self.right[0].shape[0])

    @property
    def npairs(self) -> int:
        """Same-spin (target, occupied partner) pairs for one spin channel."""
        p = self.nk * self.nband
        return p * p

    def replace(self, **kw) -> "Workload":
        return dataclasses.replace(self, **kw)


def rpa_A(omega: float, nelec: int) -> float:
    """RPA long-range amplitude sqrt(Omega / (4 pi N)) of the Jastrow function."""
    return math.sqrt(omega / (4.0 * math.pi * nelec))


def cusp_C(A: float):
    """Parallel / antiparallel lengths from the approximate cusp condition."""
    return (math.sqrt(2.0 * A), math.sqrt(A))


def _orthonormal_random(rng, npw, nb, envelope):
    z = rng.standard_normal((npw, nb)) + 1j * rng.standard_normal((npw, nb))
    z *= envelope[:, None]
    q, r = np.linalg.qr(z)
    # fix the phase convention so that R has a positive diagonal
    d = np.diag(r)
    q = q * (d / np.abs(d))[None, :]
    return np.ascontiguousarray(q.T)


def random_orbitals(lattice, kmesh, ecut, nb, sigma, seed, left_mix=None, kshift=(0.0, 0.0, 0.0)):
    B = reciprocal(lattice)
    rng = np.random.Generator(np.random.PCG64(seed))
    mill, right, left = [], [], []
    for kf in kmesh_fractions(*kmesh, shift=kshift):
        M = miller_sphere(lattice, kf, ecut)
        G = M @ B
        env = np.exp(-np.sum(G * G, axis=1) / (2.0 * sigma * sigma))
        mill.append(M)
        right.append(_orthonormal_random(rng, M.shape[0], nb, env))
        if left_mix is not None:
            z = rng.standard_normal((nb, M.shape[0])) + 1j * rng.standard_normal((nb, M.shape[0]))
            z *= env[None, :]
            z /= np.linalg.norm(z, axis=1, keepdims=True)
            left.append(right[-1] + left_mix * z)
    return mill, right, (left if left_mix is not None else None)


def perturbed_start(w, amp, seed, left_amp=None):
    """An SCF starting point: each k-point's orbitals plus amp times random complex noise on its plane-wave
    set, orthonormalised (QR); with left_amp, also a left set = right + left_amp noise (biorthogonal mode)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    right, left = [], []
    for c in w.right:
        z = rng.standard_normal(c.shape) + 1j * rng.standard_normal(c.shape)
        q, r = np.linalg.qr((c + amp * z / np.sqrt(c.shape[1])).T)
        q = q * (np.diag(r) / np.abs(np.diag(r)))[None, :]
        right.append(np.ascontiguousarray(q.T))
        if left_amp is not None:
            z2 = rng.standard_normal(c.shape) + 1j * rng.standard_normal(c.shape)
            left.append(right[-1] + left_amp * z2 / np.sqrt(c.shape[1]))
    return w.replace(right=right, left=left if left_amp is not None else None)


def polarized(w, seed, mix=0.3, occ_dn=None):
    """A spin-polarised variant: the down channel's orbitals are the up ones rotated by a random unitary
    mixing with other random smooth vectors of the same plane-wave sets (orthonormal), with fillings
    occ_dn (default: the up fillings); a left set for the down channel when the workload has one."""
    rng = np.random.Generator(np.random.PCG64(seed))
    rd, ld = [], []
    for ik, c in enumerate(w.right):
        z = rng.standard_normal(c.shape) + 1j * rng.standard_normal(c.shape)
        env = np.abs(c).max(axis=0) + 1e-3
        q, r = np.linalg.qr((c + mix * z * env[None, :] / np.linalg.norm(env)).T)
        q = q * (np.diag(r) / np.abs(np.diag(r)))[None, :]
        rd.append(np.ascontiguousarray(q.T))
        if w.left is not None:
            z2 = rng.standard_normal(c.shape) + 1j * rng.standard_normal(c.shape)
            ld.append(rd[-1] + 0.1 * z2 / np.sqrt(c.shape[1]))
    od = [np.asarray(o, dtype=np.float64).copy() for o in w.occ] if occ_dn is None else \
        [np.asarray(occ_dn, dtype=np.float64) for _ in w.occ]
    return w.replace(right_dn=rd, left_dn=ld if w.left is not None else None, occ_dn=od,
                     name=w.name + "_pol")


# --------------------------------------------------------------------------
# Crystal symmetry of the synthetic cells.  An operation {R | tau} maps fractional positions
# x -> R (x + tau) (R integer, acting on lattice coordinates); k-point k0 maps to R^T k0 - b with b
# integer such that the image lies in the mesh cell.  The orbital of the image is generated as
# c_k(m) = c_k0(m0) exp(2 pi i (m - b).tau), m = R^T m0 + b (the convention of the C ABI).
# --------------------------------------------------------------------------

def _signed_permutations():
    out = []
    for perm in ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)):
        for signs in range(8):
            S = np.zeros((3, 3))
            for i in range(3):
                S[i, perm[i]] = -1.0 if (signs >> i) & 1 else 1.0
            out.append(S)
    return out


def point_group_ops(lattice, cartesian=None):
    """Integer matrices R (x -> R x, fractional) of the cubic rotations S (Cartesian) that map the lattice
    onto itself, identity first; ``cartesian`` restricts S to a given list."""
    L = np.asarray(lattice, dtype=np.float64)
    Ss = _signed_permutations() if cartesian is None else cartesian
    ops = []
    for S in Ss:
        R = np.linalg.inv(L.T) @ S @ L.T
        Ri = np.rint(R)
        if np.max(np.abs(R - Ri)) < 1e-9:
            ops.append(Ri.astype(np.int32))
    ops.sort(key=lambda R: (not np.array_equal(R, np.eye(3, dtype=np.int32)), R.tobytes()))
    return ops


def symmorphic_ops(lattice):
    """(R, tau = 0) for the lattice's cubic point group (48 operations for the fcc and sc cells)."""
    return [(R, np.zeros(3)) for R in point_group_ops(lattice)]


def diamond_ops(lattice):
    """The 48 operations of the diamond structure on the fcc lattice (atoms at 0 and (1/4,1/4,1/4) in
    fractional coordinates): the 24 of T_d with tau = 0 and the 24 products with the inversion through the
    bond centre, x -> -R x + w, w = (1/4,1/4,1/4), written as R' (x + tau) with R' = -R, tau = R'^-1 w."""
    td = [S for S in _signed_permutations() if round(np.prod([S[i, np.argmax(np.abs(S[i]))] for i in range(3)])) == 1]
    ops = [(R, np.zeros(3)) for R in point_group_ops(lattice, td)]
    w = np.array([0.25, 0.25, 0.25])
    for R, _ in list(ops):
        Rp = -R
        ops.append((Rp.astype(np.int32), np.linalg.solve(Rp.astype(np.float64), w)))
    return ops


def _map_k(R, kf, kmesh):
    g = R.T @ kf
    t = np.rint(g * np.asarray(kmesh)).astype(int)
    assert np.max(np.abs(g * np.asarray(kmesh) - t)) < 1e-9, "operation does not map the mesh"
    idx = np.mod(t, kmesh)
    b = (t - idx) // np.asarray(kmesh)
    return int((idx[0] * kmesh[1] + idx[1]) * kmesh[2] + idx[2]), b


def k_orbits(ops, kmesh):
    """Representative (lowest index of the orbit), operation index (-1 for a representative) and b for
    every mesh k-point; the first listed operation that carries the representative onto k is used."""
    kf = kmesh_fractions(*kmesh)
    nk = len(kf)
    rep, opi, bb = [-1] * nk, [-1] * nk, [np.zeros(3, int)] * nk
    for k in range(nk):
        if rep[k] >= 0:
            continue
        rep[k] = k
        for o, (R, _) in enumerate(ops):
            kk, b = _map_k(R, kf[k], kmesh)
            if rep[kk] < 0:
                rep[kk], opi[kk], bb[kk] = k, o, b
    return rep, opi, bb


def image_map(R, tau, b, miller_from, miller_to):
    """(g0, phase) with coefficient g of the image = phase[g] * coefficient g0[g] of the source."""
    look = {tuple(m): i for i, m in enumerate(np.asarray(miller_from))}
    Rit = np.rint(np.linalg.inv(R.astype(np.float64)).T).astype(int)
    g0 = np.empty(len(miller_to), dtype=np.int64)
    ph = np.empty(len(miller_to), dtype=np.complex128)
    for g, m in enumerate(np.asarray(miller_to)):
        mb = m - b
        g0[g] = look[tuple(Rit @ mb)]
        ph[g] = np.exp(2j * math.pi * float(mb @ tau))
    return g0, ph


def symmetric_orbitals(w, ops, seed, strength=0.5, tries=50):
    """Orbitals invariant under ``ops``: at each representative k-point the nb lowest eigenvectors of a
    random Hermitian matrix (|k+G|^2/2 plus smooth random couplings) averaged over the operations that fix
    the k-point, with a gap above the nb-th eigenvalue and wherever the filling changes (closed sets); the
    other k-points' orbitals are
    the images under the first operation carrying their representative onto them."""
    rep, opi, bb = k_orbits(ops, w.kmesh)
    kf = w.kfrac
    B = reciprocal(w.lattice)
    nb = w.nband
    right = [None] * w.nk
    rng = np.random.Generator(np.random.PCG64(seed))
    for r in sorted(set(rep)):
        M = np.asarray(w.miller[r])
        n = M.shape[0]
        little = []
        for R, tau in ops:
            kk, b = _map_k(R, kf[r], w.kmesh)
            if kk == r:
                g0, ph = image_map(R, tau, b, M, M)
                O = np.zeros((n, n), dtype=np.complex128)
                O[np.arange(n), g0] = ph
                little.append(O)
        kg = (M + kf[r][None, :]) @ B
        t = 0.5 * np.sum(kg * kg, 1)
        env = np.exp(-0.25 * t)
        for _ in range(tries):
            X = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
            H = np.diag(t) + strength * (X + X.conj().T) * np.outer(env, env)
            Hs = sum(O @ H @ O.conj().T for O in little) / len(little)
            ev, V = np.linalg.eigh(Hs)
            # gaps above the set and wherever the filling changes inside it (bands of one filling closed)
            f = np.asarray(w.occ[r], dtype=np.float64)
            cuts = [nb] + [i for i in range(1, nb) if f[i] != f[i - 1]]
            if all(ev[i] - ev[i - 1] > 1e-6 * max(1.0, abs(ev[i])) for i in cuts):
                break
        else:
            raise RuntimeError(f"no closed set of {nb} bands at k-point {r}")
        right[r] = np.ascontiguousarray(V[:, :nb].T)
    for k in range(w.nk):
        if rep[k] == k:
            continue
        R, tau = ops[opi[k]]
        g0, ph = image_map(R, tau, bb[k], w.miller[rep[k]], w.miller[k])
        right[k] = np.ascontiguousarray(right[rep[k]][:, g0] * ph[None, :])
    occ = [np.asarray(w.occ[rep[k]], dtype=np.float64).copy() for k in range(w.nk)]
    return w.replace(right=right, left=None, occ=occ, name=w.name + "_sym")


def sym_arrays(ops):
    """(rot [nsym][3][3] int32, tau [nsym][3] float64) as the C ABI takes them."""
    rot = np.ascontiguousarray(np.stack([R for R, _ in ops]).astype(np.int32))
    tau = np.ascontiguousarray(np.stack([np.asarray(t, dtype=np.float64) for _, t in ops]))
    return rot, tau


def with_band(w, kpoints, seed=None, source=None, shift=None, nb=None, ecut=None, occ=None):
    """Adds band k-points (fractional, any position) to a workload.  Orbitals: with ``source`` (a mesh
    k index per band k-point) the source k-point's coefficients on its own plane-wave set, shifted by the
    integer vector ``shift`` (m -> m - shift, for k = k_source + shift + small offset); otherwise random
    smooth orthonormal orbitals (seeded) on the sphere |k + G|^2 / 2 <= ecut.  Fillings ``occ`` per band
    (default: those of the source, or 1)."""
    kpoints = np.asarray(kpoints, dtype=np.float64).reshape(-1, 3)
    B = reciprocal(w.lattice)
    rng = np.random.Generator(np.random.PCG64(SEED_BASE + 900 if seed is None else seed))
    mill, right, occs = [], [], []
    for i, kf in enumerate(kpoints):
        if source is not None:
            s0 = source[i]
            sh = np.zeros(3, dtype=np.int32) if shift is None else np.asarray(shift[i], dtype=np.int32)
            mill.append((np.asarray(w.miller[s0]) - sh[None, :]).astype(np.int32))
            right.append(np.array(w.right[s0], dtype=np.complex128))
            occs.append(np.asarray(w.occ[s0] if occ is None else occ, dtype=np.float64).copy())
        else:
            M = miller_sphere(w.lattice, kf, ecut)
            G = (M + kf[None, :]) @ B
            env = np.exp(-np.sum(G * G, axis=1) / (2.0 * (3.0 * 2.0 * math.pi / 10.26) ** 2))
            n = w.nband if nb is None else nb
            mill.append(M)
            right.append(_orthonormal_random(rng, M.shape[0], n, env))
            occs.append(np.ones(n) if occ is None else np.asarray(occ, dtype=np.float64))
    return w.replace(band_k=kpoints, band_miller=mill, band_right=right, band_occ=occs)


def grid_fits(miller_list, grid) -> bool:
    """True when every pair density is alias-free: N_i/2 >= 2 max|m_i| + 1."""
    mx = np.max(np.stack([np.max(np.abs(m), axis=0) for m in miller_list]), axis=0)
    return all(grid[i] // 2 >= 2 * mx[i] + 1 for i in range(3))


# --------------------------------------------------------------------------
# Named workloads.  Geometry follows the paper's examples (simple-cubic
# electron gas; fcc diamond-lattice silicon cell a = 10.26 bohr); everything
# else is synthetic.
# --------------------------------------------------------------------------

def heg_gamma(rs=4.0, nelec=14, grid=16, mmax2=9, occ_m2=1) -> Workload:
    """Electron gas, Gamma only: occupied shell |m|^2 <= occ_m2 (7 plane waves for 14 electrons)."""
    L = (nelec * 4.0 * math.pi / 3.0 * rs ** 3) ** (1.0 / 3.0)
    lat = sc_lattice(L)
    M = miller_norm2(mmax2)
    occm = miller_norm2(occ_m2)
    nb = occm.shape[0]
    coef = np.zeros((nb, M.shape[0]), dtype=np.complex128)
    for b, m in enumerate(occm):
        idx = np.where(np.all(M == m[None, :], axis=1))[0][0]
        coef[b, idx] = 1.0
    A = rpa_A(L ** 3, nelec)
    kc = 3.0 * 2.0 * math.pi / L
    return Workload("heg14_gamma", lat, (1, 1, 1), (grid,) * 3, [M], [coef], None,
                    [np.ones(nb)], (A, A), cusp_C(A), 10.0 / kc ** 2, nelec)


def heg_twist(rs=2.0, nelec=54, tw=2, grid=32, ecut=None, nocc=27, kshift=(0.0, 0.0, 0.0)) -> Workload:
    """Electron gas on a tw^3 twist grid (shifted by ``kshift`` mesh units); nocc lowest |k+G|^2 plane waves
    per twist."""
    L = (nelec * 4.0 * math.pi / 3.0 * rs ** 3) ** (1.0 / 3.0)
    lat = sc_lattice(L)
    if ecut is None:
        ecut = 5.78
    mill, right = [], []
    for kf in kmesh_fractions(tw, tw, tw, shift=kshift):
        M = miller_sphere(lat, kf, ecut)             # sorted by |k+G|^2 then m
        coef = np.zeros((nocc, M.shape[0]), dtype=np.complex128)
        coef[np.arange(nocc), np.arange(nocc)] = 1.0
        mill.append(M)
        right.append(coef)
    A = rpa_A(L ** 3, nelec)
    kc = math.sqrt(2.0 * ecut)
    return Workload(f"heg{nelec}_twist{tw}", lat, (tw,) * 3, (grid,) * 3, mill, right, None,
                    [np.ones(nocc) for _ in mill], (A, A), cusp_C(A), 10.0 / kc ** 2, nelec,
                    kshift=tuple(float(x) for x in kshift))


def fcc_si(kmesh=(4, 4, 4), grid=24, ecut=8.14, nb=4, a=10.26, supercell=1,
           seed_offset=2, left_mix=None, occ=None, kshift=(0.0, 0.0, 0.0)) -> Workload:
    """Diamond-lattice silicon-like cell with random smooth orthonormal orbitals (k-mesh shifted by
    ``kshift`` mesh units)."""
    lat = fcc_lattice(a) * supercell
    nelec = 8 * supercell ** 3
    omega = abs(np.linalg.det(lat))
    sigma = 3.0 * 2.0 * math.pi / a
    mill, right, left = random_orbitals(lat, kmesh, ecut, nb, sigma,
                                        SEED_BASE + seed_offset, left_mix, kshift)
    A = rpa_A(omega, nelec)
    kc = math.sqrt(2.0 * ecut)
    nk = int(np.prod(kmesh))
    occs = [np.ones(nb) if occ is None else np.asarray(occ, dtype=np.float64) for _ in range(nk)]
    return Workload(f"fcc_si_x{supercell}_k{'x'.join(map(str, kmesh))}_g{grid}",
                    lat, tuple(kmesh), (grid,) * 3 if np.isscalar(grid) else tuple(grid),
                    mill, right, left, occs, (A, A), cusp_C(A), 10.0 / kc ** 2, nelec,
                    kshift=tuple(float(x) for x in kshift))


WORKLOADS = {
    # 14-electron gas at r_s = 4, Gamma only, 7 occupied plane waves, 16^3 grid (49 pairs)
    "heg14_g16": heg_gamma,
    # fcc a = 10.26 bohr, 4x4x4 k-mesh, 4 bands, ~300 plane waves, 24^3 grid (65,536 pairs)
    "fcc_si_k444_g24": fcc_si,
    # 54-electron gas at r_s = 2, 2x2x2 twists, 27 bands, 32^3 grid (46,656 pairs)
    "heg54_twist2_g32": heg_twist,
    # 2x2x2 supercell of the fcc cell, 2x2x2 k-mesh, 32 bands, ~2400 plane waves, 48^3 grid (65,536 pairs)
    "fcc_si_x2_k222_g48": lambda: fcc_si(kmesh=(2, 2, 2), grid=48, nb=32, supercell=2, seed_offset=4),
    # the fcc bench shape in the biorthogonal mode: left orbitals chi = phi + 0.1 z (z random, same
    # envelope, unit norm), biorthogonalised by the consumer
    "fcc_si_k444_g24_bitc": lambda: fcc_si(left_mix=0.1).replace(name="fcc_si_x1_k4x4x4_g24_bitc"),
    # the fcc bench shape with orbitals invariant under the diamond structure's 48 operations (8 of the
    # 64 k-points are representatives)
    "fcc_si_k444_g24_sym": lambda: symmetric_orbitals(fcc_si(), diamond_ops(fcc_lattice(10.26)), SEED_BASE + 44),
    # the fcc bench shape with 16 band k-points on the path L - Gamma - X (none on the 4x4x4 mesh), four
    # random smooth orbitals each on their own plane-wave sets
    "fcc_si_k444_g24_band16": lambda: with_band(fcc_si(), band_path_fcc(), seed=SEED_BASE + 45, ecut=8.14, nb=4),
}


def band_path_fcc():
    """16 fractional k-points on L - Gamma - X of the fcc reciprocal lattice (L = (1/2,1/2,1/2), X = (1/2,1/2,0)
    in units of the reciprocal rows), avoiding the 4x4x4 mesh."""
    L = np.array([0.5, 0.5, 0.5])
    X = np.array([0.5, 0.5, 0.0])
    s = [0.05, 0.17, 0.29, 0.41, 0.53, 0.65, 0.77, 0.89]
    return np.array([L * (1.0 - t) for t in s] + [X * t for t in [0.11, 0.23, 0.37, 0.47, 0.61, 0.73, 0.83, 0.97]])


def workload(name: str) -> Workload:
    """A named full-size workload (see WORKLOADS)."""
    return WORKLOADS[name]()


def tiny_fcc(kmesh=(2, 1, 1), grid=8, ecut=1.2, nb=2, a=6.0, seed_offset=100,
             left_mix=None, occ=None, A=None, C=None, alpha=None, kshift=(0.0, 0.0, 0.0)) -> Workload:
    """A small random problem the oracle finishes in well under a second."""
    w = fcc_si(kmesh=kmesh, grid=grid, ecut=ecut, nb=nb, a=a, seed_offset=seed_offset,
               left_mix=left_mix, occ=occ, kshift=kshift)
    repl = {"name": f"tiny_fcc_k{'x'.join(map(str, kmesh))}_g{grid}"}
    if A is not None:
        repl["A"] = tuple(A)
    if C is not None:
        repl["C"] = tuple(C)
    if alpha is not None:
        repl["alpha"] = alpha
    return w.replace(**repl)
