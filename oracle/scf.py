"""Oracle O5: the TC / BITC self-consistent loop by exact diagonalisation in the plane-wave basis.

TEST INFRASTRUCTURE ONLY (imported by tests/ alone).  NumPy / PyTorch CPU, complex128.

Sec. 2.4 writes the SCF equation as the eigenvalue problem of the non-Hermitian one-body operator
T + h[phi] (Eq. SCF; Eq. BITCSCF with left orbitals), whose operator depends on the occupied orbitals
and is updated as they change.  Each iteration here:
  1. builds the full matrix of T + h[phi_occ] on every k-point's plane-wave set.  h is applied to every
     unit vector e_G by the FFT-route oracle O1, with the unit vectors added to the orbital set as bands
     of zero filling: they are then targets of every term and partners of none (every partner sum is
     weighted by the filling), so their output rows are h e_G;
  2. diagonalises each matrix (numpy.linalg.eig) and keeps the nband eigenvectors of lowest real
     eigenvalue;
  3. TC: orthonormalises them in eigenvalue order (Gram-Schmidt, Sec. 2.3); BITC: takes the right
     eigenvectors as phi and the left ones as chi and biorthonormalises the pair (Sec. 2.3: the
     eigenvectors of distinct eigenvalues are already biorthogonal);
  4. evaluates the energy (reading R8) of the orbital set that defines the next operator;
until the energy changes by less than etol.  The fillings stay fixed.

davidson_scf follows the block-Davidson steps of Sec. 2.4 instead of the exact diagonalisation, with
the operator applied through the same full matrices: its iterates are those of the library's loop.

Density-matrix mixing (Sec. 2.4) with ratio beta < 1: the operator and the energy of an iteration use
the new orbitals with fillings beta f together with the previous iteration's orbitals, as extra bands,
with fillings (1 - beta) f.  The eigenvectors are taken for the new orbitals only.  The returned
orbitals are the last new ones; the final energy is evaluated for them alone.
"""
from __future__ import annotations

import numpy as np
import torch

from .fftroute import ALL_TERMS, MULT, Problem, biorthogonalize_coeffs


def _kinetic_diag(w, k):
    B = 2.0 * np.pi * np.linalg.inv(np.asarray(w.lattice, dtype=np.float64)).T
    kg = (w.kfrac[k][None, :] + np.asarray(w.miller[k])) @ B
    return 0.5 * np.sum(kg * kg, 1)


def operator_matrices(w, right, left=None, terms=ALL_TERMS, reading="printed", spin=0, right_dn=None):
    """[T + h[phi]] on each k-point's plane-wave set, H[k][G', G] = <e_G'| T + h |e_G>.

    ``right``/``left``: per k (nb, npw) arrays, used as given (left already biorthonormal, or None);
    ``reading``: the mesh corrections' reading of the FFT-route oracle (R4).  Spin-polarised workloads
    (TC mode): ``right_dn`` the down channel's orbitals (default the workload's), ``spin`` the channel
    whose operator is returned; the unit vectors join both channels with zero filling.
    """
    nk = w.nk
    npw = [m.shape[0] for m in w.miller]
    nx = max(npw)
    pol = getattr(w, "right_dn", None) is not None
    dn = (w.right_dn if right_dn is None else right_dn) if pol else None
    ext_r, ext_l, occ, ext_d, occ_d = [], [], [], [], []
    for k in range(nk):
        E = np.zeros((nx, npw[k]), dtype=np.complex128)
        E[np.arange(npw[k]), np.arange(npw[k])] = 1.0
        ext_r.append(np.concatenate([right[k], E]))
        if left is not None:
            ext_l.append(np.concatenate([left[k], E]))
        occ.append(np.concatenate([np.asarray(w.occ[k], dtype=np.float64), np.zeros(nx)]))
        if pol:
            ext_d.append(np.concatenate([dn[k], E]))
            od = w.occ_dn if w.occ_dn is not None else w.occ
            occ_d.append(np.concatenate([np.asarray(od[k], dtype=np.float64), np.zeros(nx)]))
    if pol:
        wx = w.replace(right=ext_r, left=None, occ=occ, right_dn=ext_d, left_dn=None, occ_dn=occ_d)
    else:
        wx = w.replace(right=ext_r, left=ext_l if left is not None else None, occ=occ)
    pr = Problem(wx, biorthogonalize=False, reading=reading)
    g = sum(MULT.get(t, 1) * pr.term(t, spin) for t in terms)
    hc = pr.to_coeff(g, spin)
    nb = right[0].shape[0]
    out = []
    for k in range(nk):
        rows = hc[k][nb:nb + npw[k]].numpy()            # rows: h e_G on the plane-wave set
        out.append(rows.T + np.diag(_kinetic_diag(w, k)))
    return out


def _gram_schmidt(V):
    """Columns of V orthonormalised in order (classical Gram-Schmidt with one re-orthogonalisation)."""
    Q = np.array(V, dtype=np.complex128)
    for j in range(Q.shape[1]):
        for _ in range(2):
            for i in range(j):
                Q[:, j] -= np.vdot(Q[:, i], Q[:, j]) * Q[:, i]
        Q[:, j] /= np.linalg.norm(Q[:, j])
    return Q


def energy(w, right, left=None):
    """Energy per cell of the given orbitals (left used as given)."""
    wx = w.replace(right=list(right), left=list(left) if left is not None else None)
    return float(Problem(wx, biorthogonalize=False).energy())


def _mixed(w, right, left, old_r, old_l, beta):
    """Orbital set of the operator: new orbitals (beta f) and previous ones ((1 - beta) f)."""
    if old_r is None or beta >= 1.0:
        return w, right, left
    occ = [np.concatenate([beta * np.asarray(o, float), (1.0 - beta) * np.asarray(o, float)]) for o in w.occ]
    r = [np.concatenate([a, b]) for a, b in zip(right, old_r)]
    l = None if left is None else [np.concatenate([a, b]) for a, b in zip(left, old_l)]
    return w.replace(occ=occ), r, l


def scf(w, max_iter=60, etol=1e-11, mix=1.0):
    """Returns (energies per iteration, right, left or None, orbital eigenvalues per k, final energy)."""
    bitc = w.left is not None
    if bitc:
        cr, cl = biorthogonalize_coeffs([torch.as_tensor(c) for c in w.right], [torch.as_tensor(c) for c in w.left])
        right, left = [c.numpy() for c in cr], [c.numpy() for c in cl]
    else:
        right, left = [np.asarray(c, dtype=np.complex128) for c in w.right], None
    nb = right[0].shape[0]
    hist, evals = [], None
    old_r = old_l = None
    wm, mr, ml = w, right, left
    for _ in range(max_iter):
        H = operator_matrices(wm, mr, ml)
        new_r, new_l, evals = [], [], []
        for k, Hk in enumerate(H):
            lam, VR = np.linalg.eig(Hk)
            idx = np.argsort(lam.real, kind="stable")[:nb]
            evals.append(lam[idx])
            if bitc:
                VL = np.linalg.inv(VR).conj().T                  # columns: left eigenvectors
                r = VR[:, idx].T
                l = VL[:, idx].T
                cr, cl = biorthogonalize_coeffs([torch.as_tensor(r)], [torch.as_tensor(l)])
                new_r.append(cr[0].numpy())
                new_l.append(cl[0].numpy())
            else:
                new_r.append(_gram_schmidt(VR[:, idx]).T)
        old_r, old_l = right, left
        right, left = new_r, (new_l if bitc else None)
        wm, mr, ml = _mixed(w, right, left, old_r, old_l, mix)
        hist.append(energy(wm, mr, ml))
        if len(hist) > 1 and abs(hist[-1] - hist[-2]) < etol:
            break
    return hist, right, left, evals, energy(w, right, left)


def _payne(x):
    """Preconditioner of Payne et al. (Sec. 2.4) as a function of x."""
    num = 27.0 + 18.0 * x + 12.0 * x ** 2 + 8.0 * x ** 3
    return num / (num + 16.0 * x ** 4)


def _gs_append(cols, v, atol=1e-8, rtol=1e-8):
    """Orthonormalise v against the columns kept so far; None when it is negligible or dependent."""
    n0 = np.linalg.norm(v)
    if n0 < atol:
        return None
    u = np.array(v, dtype=np.complex128)
    for _ in range(2):
        for c in cols:
            u -= np.vdot(c, u) * c
    n = np.linalg.norm(u)
    if not n > rtol * n0:
        return None
    return u / n


def davidson_scf(w, max_iter=60, pmax=2, etol=1e-11, mix=1.0):
    """Block-Davidson TC / BITC SCF (Sec. 2.4, Eq. blockDavid), one subspace diagonalisation per
    iteration with the operator updated every iteration (with mix < 1 from the mixed orbital set).
    Returns (energies per iteration, right, left, final energy of the returned orbitals alone)."""
    bitc = w.left is not None
    if bitc:
        cr, cl = biorthogonalize_coeffs([torch.as_tensor(c) for c in w.right], [torch.as_tensor(c) for c in w.left])
        right, left = [c.numpy() for c in cr], [c.numpy() for c in cl]
    else:
        right, left = [np.asarray(c, dtype=np.complex128) for c in w.right], None
    nb = right[0].shape[0]
    hist = []
    wm, mr, ml = w, right, left
    for _ in range(max_iter):
        H = operator_matrices(wm, mr, ml)
        new_r, new_l = [], []
        for k, Hk in enumerate(H):
            tG = _kinetic_diag(w, k)
            cols = []
            for i in range(nb):                         # block 0: the current right orbitals
                u = _gs_append(cols, right[k][i])
                if u is not None:
                    cols.append(u)
            blocks = [list(range(len(cols)))]
            eps = [np.vdot(cols[i], Hk @ cols[i]) for i in range(nb)] if len(cols) == nb else None
            prev = [cols[i] for i in range(nb)]
            for _p in range(pmax):
                nxt = []
                for i in range(nb):
                    v = prev[i]
                    if v is None:
                        nxt.append(None)
                        continue
                    t = np.sum(tG * np.abs(v) ** 2)
                    x = tG / t if t > 0 else np.zeros_like(tG)
                    res = Hk @ v - eps[i] * v
                    # reading: the 'very small norm' (< 1e-8) test of Sec. 2.4 is applied to the residual
                    # before preconditioning; the preconditioner can shrink it by orders of magnitude when
                    # the vector's kinetic energy t is small
                    u = None if np.linalg.norm(res) < 1e-8 else _gs_append(cols, _payne(x) * res, atol=0.0)
                    if u is not None:
                        cols.append(u)
                    nxt.append(u if u is not None else np.zeros_like(v))
                prev = nxt
            Vm = np.stack(cols, 1)
            Hs = Vm.conj().T @ Hk @ Vm
            lam, VR = np.linalg.eig(Hs)
            idx = np.argsort(lam.real, kind="stable")[:nb]
            phi = Vm @ VR[:, idx]
            if bitc:
                VL = np.linalg.inv(VR).conj().T
                chi = Vm @ VL[:, idx]
                cr, cl = biorthogonalize_coeffs([torch.as_tensor(phi.T)], [torch.as_tensor(chi.T)])
                new_r.append(cr[0].numpy())
                new_l.append(cl[0].numpy())
            else:
                new_r.append(_gram_schmidt(phi).T)
        old_r, old_l = right, left
        right, left = new_r, (new_l if bitc else None)
        wm, mr, ml = _mixed(w, right, left, old_r, old_l, mix)
        hist.append(energy(wm, mr, ml))
        if len(hist) > 1 and abs(hist[-1] - hist[-2]) < etol:
            break
    return hist, right, left, energy(w, right, left)
