"""Oracle O3: closed forms for plane-wave orbitals (homogeneous electron gas).

TEST INFRASTRUCTURE ONLY.  NumPy float64, no grid and no FFT.  When every
occupied orbital is a single plane wave e^{i p.r} (p = k + G), every pair
density has one Fourier component, FT[chi*_q phi_j] = delta_{G, G_j - G_q}/Omega,
so each term of Sec. 2.6 is diagonal, g_j = eps_j phi_j, with eps_j a finite
sum over occupied momenta of the analytic kernels (Sec. 2.6.3, Appendix B).
Densities are uniform, so every Hartree-type term (2ah, 2bh1, 2bh2, 3a1, 3a3,
3b1, 3b2, 3b3) vanishes (G = 0 is dropped).  Valid while the FFT grid does not
alias the pair densities.  Kernel values at Q = 0 follow the same readings as
the FFT-route oracle; the divergence corrections are the SCF-mesh ones, whose
G != 0 parts vanish for plane waves.
"""
from __future__ import annotations

import math

import numpy as np

FOURPI = 4.0 * math.pi


def _kern(P, A, C):
    """(u~, lap-u~, (grad u)^2~, 4pi/Q^2) at the cartesian vectors P (n,3); Q = 0 rows use exchange limits."""
    Q2 = np.sum(P * P, axis=-1)
    zero = Q2 < 1e-20
    Q2s = np.where(zero, 1.0, Q2)
    ic2 = 1.0 / C ** 2
    ut = FOURPI * A * (1.0 / Q2s - 1.0 / (Q2s + ic2))
    lap = -FOURPI * A * ic2 / (Q2s + ic2)
    g = C * np.sqrt(Q2s)
    W = FOURPI * A * A / (C * g) * (-math.pi * g * g / 4.0 - (1 + g * g / 2) * np.arctan(g / 2)
                                      + (1 + g * g) * np.arctan(g))
    v = FOURPI / Q2s
    ut = np.where(zero, 0.0, ut)
    lap = np.where(zero, -FOURPI * A, lap)
    W = np.where(zero, 2.0 * math.pi * A * A / C, W)
    v = np.where(zero, 0.0, v)
    return ut, lap, W, v


def gb_delta(lattice, kmesh, alpha):
    """Gygi-Baldereschi bracket of Eq. correction2 (ball exp(-alpha q^2) > 1e-18)."""
    lat = np.asarray(lattice, dtype=np.float64)
    B = 2.0 * math.pi * np.linalg.inv(lat).T
    omega = abs(np.linalg.det(lat))
    n1, n2, n3 = kmesh
    nk = n1 * n2 * n3
    qmax = math.sqrt(41.45 / alpha)
    mm = [int(math.ceil(qmax * np.linalg.norm(a) / (2 * math.pi))) + 2 for a in lat]
    rr = [np.arange(-m, m + 1) for m in mm]
    M = np.stack(np.meshgrid(*rr, indexing="ij"), -1).reshape(-1, 3)
    tot = 0.0
    for i1 in range(n1):
        for i2 in range(n2):
            for i3 in range(n3):
                q = np.array([i1 / n1, i2 / n2, i3 / n3])
                Q = (M - q) @ B
                q2 = np.sum(Q * Q, 1)
                ok = (q2 > 1e-20) & (alpha * q2 < 41.45)
                tot += math.fsum(np.exp(-alpha * q2[ok]) / q2[ok])
    return omega / (4.0 * math.sqrt(math.pi ** 3 * alpha)) - (-alpha + tot) / nk


def heg_terms(w, A=None, C=None, alpha=None, div_correction=True, reading="printed"):
    """Diagonal eigenvalue of every printed term for every occupied plane wave.

    Returns (eps, momenta, weights) with eps[term] an array over orbitals of one
    spin channel (both channels are equal for unpolarized input).  Bands of zero
    filling are targets of every term and partners of none; a target's divergence
    corrections take the filling of the occupied plane wave of the same momentum
    (FT[phi*_mu phi_j](0) = delta_{p_mu, p_j}/Omega).  ``reading``
    selects the mesh corrections as in the FFT-route oracle: "printed" (one
    u~_short(0)/N_k in the G = G' = 0 corrections of 3a2 and 3b6, no 2bx1 mesh
    correction) or "limit" (two, and the 2bx1 remainder -(4 pi A_par / N_k) f_j / Omega).
    """
    if reading not in ("printed", "limit"):
        raise ValueError("reading must be 'printed' or 'limit'")
    um = 1.0 if reading == "printed" else 2.0
    lat = np.asarray(w.lattice, dtype=np.float64)
    B = 2.0 * math.pi * np.linalg.inv(lat).T
    omega = abs(np.linalg.det(lat))
    nk = int(np.prod(w.kmesh))
    n1, n2, n3 = w.kmesh
    s1, s2, s3 = (float(x) for x in getattr(w, "kshift", (0.0, 0.0, 0.0)))   # Monkhorst-Pack shift
    kf = [np.array([(i1 + s1) / n1, (i2 + s2) / n2, (i3 + s3) / n3])
          for i1 in range(n1) for i2 in range(n2) for i3 in range(n3)]
    A = np.asarray(w.A if A is None else A, dtype=np.float64)
    C = np.asarray(w.C if C is None else C, dtype=np.float64)
    alpha = w.alpha if alpha is None else alpha
    ps, fs = [], []
    for ik in range(nk):
        for b in range(w.right[ik].shape[0]):
            c = w.right[ik][b]
            i = int(np.argmax(np.abs(c)))
            assert abs(abs(c[i]) - 1.0) < 1e-12, "plane-wave orbitals required"
            ps.append((kf[ik] + w.miller[ik][i]) @ B)
            fs.append(float(w.occ[ik][b]))
    p = np.array(ps)
    f = np.array(fs)
    wq = f / nk
    P = p.shape[0]
    dgb = gb_delta(lat, w.kmesh, alpha) if div_correction else 0.0
    nbar = np.sum(wq) / omega                       # per-spin density
    ushort = -FOURPI * A * C * C
    D = p[:, None, :] - p[None, :, :]              # D[j,q] = p_j - p_q
    same = np.sum(D * D, -1) < 1e-20                # pairs of one plane wave (Q = 0)
    off = ~same
    fs = (same * f[None, :]).sum(1)                 # filling of the occupied plane wave of p_j
    K = [_kern(D.reshape(-1, 3), A[s], C[s]) for s in range(2)]
    ut = [k[0].reshape(P, P) for k in K]
    lap = [k[1].reshape(P, P) for k in K]
    W = [k[2].reshape(P, P) for k in K]
    v = K[0][3].reshape(P, P)
    V2a = v + lap[0] - W[0]
    eps = {t: np.zeros(P) for t in ("2ah", "2bh1", "2bh2", "2ax", "2bx1", "2bx2", "3a1", "3a2", "3a3",
                                      "3a4", "3b1", "3b2", "3b3", "3b4", "3b5", "3b6")}
    # 2ax: -(1/Omega) sum_q w_q V2a(p_j - p_q) (Q = 0 row keeps L(0)-W(0)) + GB
    eps["2ax"] = -(V2a * wq[None, :]).sum(1) / omega - FOURPI * dgb * fs / omega
    # 2bx1 / 2bx2
    dot_q = np.einsum("jqa,qa->jq", D, p)
    dot_j = np.einsum("jqa,ja->jq", D, p)
    eps["2bx1"] = (wq[None, :] * ut[0] * dot_q * off).sum(1) / omega
    eps["2bx2"] = -(wq[None, :] * ut[0] * dot_j * off).sum(1) / omega
    if div_correction and reading == "limit":
        eps["2bx1"] = eps["2bx1"] - FOURPI * A[0] / nk * fs / omega
    # 3a2: h5^{s,s2}(q2) = sum_{q1 != q2} w_q1 P^2 u~^2 / Omega^2 + corrections; both spins s2
    Dn2 = np.sum(D * D, -1)
    h6 = 0.0
    for s in (0, 1):                 # channel of (target spin, spin of q1 and q2)
        h5 = (wq[:, None] * Dn2 * ut[s] ** 2 * off).sum(0) / omega ** 2     # index q2 (sum over q1)
        if div_correction:
            c1 = FOURPI * A[s] * (FOURPI * A[s] * dgb + um * ushort[s] / nk)   # reading R4
            h5 = h5 + c1 * fs / omega ** 2
        h6 += np.sum(wq * h5)
    eps["3a2"] = np.full(P, 0.5 * h6)
    # vector sums a(q2) = (i/Omega) sum_{q1 != q2} w_q1 (p_q2 - p_q1) u~(p_q2 - p_q1)
    a = 1j * np.einsum("xy,xya,xy->xa", wq[None, :] * np.ones((P, P)), D, ut[0] * off) / omega
    b = a                                           # h3 of Alg. 3b4 (same sum, target index)
    c = -a                                          # H3b(q2) coefficient
    iPu = 1j * D * (ut[0] * off)[..., None]        # [j,q] -> i(p_j - p_q) u~(p_j - p_q)
    eps["3a4"] = -0.5 * np.einsum("q,qa,jqa->j", wq, a, iPu) / omega
    eps["3b4"] = 0.5 * np.einsum("q,jqa,ja->j", wq, iPu, b) / omega
    eps["3b5"] = 0.5 * np.einsum("q,jqa,qa->j", wq, iPu, c) / omega   # -1/2 of the definition times -U
    b6 = np.zeros(P)
    for s in (0, 1):                # channel of (spin of the density, target spin)
        b6 = b6 + 0.5 * (wq[None, :] * Dn2 * ut[s] ** 2 * off).sum(1) * nbar / omega
        if div_correction:
            c1 = 2.0 * math.pi * A[s] * (FOURPI * A[s] * dgb + um * ushort[s] / nk)   # reading R4
            b6 = b6 + c1 * (1.0 / omega) * nbar * fs
    eps["3b6"] = b6
    return eps, p, f


def heg_energy(w, **kw):
    """Energy per cell (both spins) from the closed forms: (1/N_k) sum f [p^2/2 + eps2/2 + eps3/3]."""
    eps, p, f = heg_terms(w, **kw)
    nk = int(np.prod(w.kmesh))
    mult = {"3a1": 1, "3a2": 1, "3a3": 2, "3a4": 2}
    parts = {"T": 2 * np.sum(f * 0.5 * np.sum(p * p, 1)).real / nk}
    for t, e in eps.items():
        fac = 0.5 if t.startswith("2") else mult.get(t, 2) / 3.0
        parts[t] = 2 * fac * np.sum(f * e).real / nk
    return sum(parts.values()), parts
