"""Oracle O1: the TC / BITC operator by the FFT pair-density route, term by term.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Plain PyTorch CPU
float64/complex128; ``torch.fft`` is used as a library primitive for the
periodic Fourier transform FT and its inverse.  Nothing is fused or reordered
beyond the paper's own algorithms; each term is computed separately.

Conventions (restating the paper's Secs. 2.2, 2.3 and 2.6 in the units used here)
  * FT[f](G) = (1/N_r) sum_r f(r) e^{-iG.r}  (periodic transform, Sec. 2.2,
    evaluated on the real-space grid), FT^{-1}[F](r) = sum_G F(G) e^{iG.r};
  * the kernels are the non-periodic transforms of Sec. 2.2 (FT(1/r) = 4pi/G^2,
    the Jastrow transforms of Sec. 2.6.3 and Appendix B);
  * a kernel applied to a Bloch pair density with crystal momentum Delta is
    sum_G K(Delta+G) FT[rho](G) e^{iG.r} (Eq. convolution), Delta = k_target -
    k_partner exactly as written in the algorithms (not reduced modulo G);
  * orbitals: physical cell-periodic parts phi(r) = Omega^{-1/2} sum c(G) e^{iG.r}
    (Secs. 2.3 and 2.6.1; the paper's dimensionless arrays are sqrt(Omega) phi and their
    1/Omega factors are restored here);
  * g_j(r) is the cell-periodic part of a term applied to phi_j, with the
    weights f_q / N_k of the algorithms.

Readings where the paper is silent or garbled:
  R1  Q = Delta+G = 0: in Hartree-type fields every kernel is dropped (Alg. 2ah
      text); in exchange-type convolutions 1/r is dropped (replaced by the GB
      correction), the Jastrow-derived scalar kernels take their finite limits
      L(0) = -4 pi A and W(0) = 2 pi A^2 / C, and the vector kernel iQu(Q) is 0.
  R2  Kernels are zero on the Nyquist planes m_i = -N_i/2 of even grids, so that
      every discrete convolution has an exact transpose (needed for an exact
      discrete adjoint); physical content never reaches those planes when the
      grid satisfies N_i/2 >= 2 max|m_i| + 1.
  R3  The 1/Omega carried by FT[chi* phi](0) is kept in every divergence
      correction (the paper's equations drop Omega factors, Sec. 2.6.1).
  R4  The mesh corrections come in two readings (``reading``):
      "printed" (default): the coefficients as printed.  The G = G' = 0
      corrections of 3a2 and 3b6 (Eqs. divcor_3a2_first, 3b6_div_scf1) carry one
      u~_short(0)/N_k, and 2bx1 has no mesh correction (the vector sum of
      Eq. correction_nabla vanishes on the mesh).
      "limit": the mesh operator is the limit of the band operator as a band
      k-point approaches a mesh point.  The G = G' = 0 corrections then carry
      2 u~_short(0)/N_k, the full finite Q -> 0 remainder of
      Q^2 u~(Q)^2 = (4 pi A / Q^2 + u~_short)(4 pi A + Q^2 u~_short); and 2bx1 gains
      the isotropic remainder -(4 pi A_par / N_k) sum_mu f_mu rho~_{mu j}(0) phi_mu
      that (nabla + ik) leaves on the partner's Bloch phase at the singular point.
      Both limits are pinned by the band forms on the CPU (tests of the band oracle).
  R13 For a band k-point the vector sum of Eq. correction_nabla is taken at the
      arguments k - q + G of the kernel it replaces (printed with q + G, which is zero
      on the mesh).
  R14 Band corrections of 3a4 and 3b5: the GB replacement is applied to the sums of
      Algs. 3a4 and 3b5 as computed, whose two i factors give i^2 = -1; the prefactors
      printed in Eqs. div_corr_3a4 and 3b5_div drop it (opposite sign).  With the
      printed sign the 1/delta divergence at k -> a mesh point doubles instead of
      cancelling.
  R5  Alg. 3b4 accumulates h2 * phi_q2 (the printed h3 <- h3 + h3 phi is a typo).
  R6  3a1 uses the bilinear h1 . h1 (printed |h1|^2; equal in TC mode).
  R7  The three-body total is 3a1 + 3a2 + 2 3a3 + 2 3a4 + 2 (3b1+...+3b6)
      (3a5 = 3a4, 3a6 = 3a3, 3c* = 3b*), checked by the brute-force oracle.
  R9  Alg. 3b5 ends with g_j <- g_j - (1/2) h5 phi_q2 f/N_k: the printed "+" contradicts
      the caption of Alg. 3b5, the term list of Sec. 2.6.4 (-1/2) and Eq. 3b5_div; the
      literal permutation integral of the brute-force oracle fixes the sign.
  R8  Energy: E = (1/N_k) Re sum_{sigma,k,mu} f <chi| T + h2/2 + h3/3 |phi> per
      cell, which equals Eq. EtotBiTC for biorthonormal determinants.
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional

import numpy as np
import torch

CD = torch.complex128
RD = torch.float64
FOURPI = 4.0 * math.pi

TERMS2 = ("2ah", "2bh1", "2bh2", "2ax", "2bx1", "2bx2")
TERMS3 = ("3a1", "3a2", "3a3", "3a4", "3b1", "3b2", "3b3", "3b4", "3b5", "3b6")
# multiplicity of each printed three-body term in the total (reading R7)
MULT = {"3a1": 1, "3a2": 1, "3a3": 2, "3a4": 2, "3b1": 2, "3b2": 2, "3b3": 2,
        "3b4": 2, "3b5": 2, "3b6": 2}
ALL_TERMS = TERMS2 + TERMS3


def _pair(s1: int, s2: int) -> int:
    """Jastrow channel: 0 = parallel spins, 1 = antiparallel."""
    return 0 if s1 == s2 else 1


def w_series(g):
    """(Cg/(4 pi A^2)) W for small g from the Taylor series of Appendix B's closed form."""
    g2 = g * g
    return 0.5 - math.pi * g / 4.0 + 11.0 * g2 / 24.0 - 57.0 * g2 * g2 / 480.0


def w_closed(g):
    """Bracket of Eq. fourier_transform_nabla2u divided by g (Appendix B)."""
    return (-math.pi * g * g / 4.0 - (1.0 + g * g / 2.0) * torch.atan(g / 2.0)
            + (1.0 + g * g) * torch.atan(g)) / g


def jastrow_kernels(Q2: torch.Tensor, A, C):
    """u~, laplacian-u~ and (grad u)^2~ of u = A/r (1 - exp(-r/C)) at |Q|^2 = Q2 > 0.

    Sec. 2.6.3: u~ = 4 pi A (1/Q^2 - 1/(Q^2 + C^-2)), (lap u)~ = -Q^2 u~,
    (grad u)^2~ = (4 pi A^2/(C g)) [-(pi/4) g^2 - (1+g^2/2) atan(g/2) + (1+g^2) atan g],
    g = C Q.  Q2 must be strictly positive (callers mask Q = 0).
    """
    ic2 = 1.0 / (C * C)
    ut = FOURPI * A * (1.0 / Q2 - 1.0 / (Q2 + ic2))
    lap = -FOURPI * A * ic2 / (Q2 + ic2)
    g = C * torch.sqrt(Q2)
    small = g < 1e-3
    gs = torch.where(small, torch.ones_like(g), g)
    br = torch.where(small, w_series(torch.where(small, g, torch.zeros_like(g))), w_closed(gs))
    W = FOURPI * A * A / C * br
    return ut, lap, W


class Problem:
    """One (possibly spin-unpolarized) TC / BITC problem on a uniform k-mesh.

    ``coeff`` / ``left`` override the workload's coefficients (per k, (nb,npw)
    complex128 torch tensors, possibly requiring grad); ``coeff_dn`` those of the
    down-spin channel of a spin-polarised workload; ``A`` / ``C`` are
    2-element float64 tensors (parallel, antiparallel), possibly requiring grad.
    Both spin channels use the same orbitals (unpolarized input).
    """

    def __init__(self, w, A=None, C=None, coeff=None, left=None, div_correction=True,
                 alpha=None, biorthogonalize=True, reading="printed", coeff_dn=None, left_dn=None):
        self.w = w
        self.lattice = np.asarray(w.lattice, dtype=np.float64)
        self.omega = abs(float(np.linalg.det(self.lattice)))
        self.B = 2.0 * math.pi * np.linalg.inv(self.lattice).T
        self.kmesh = tuple(w.kmesh)
        self.nk = int(np.prod(self.kmesh))
        n1, n2, n3 = self.kmesh
        # Monkhorst-Pack mesh with or without a shift s (mesh units): k = (i + s) / n
        self.kshift = np.asarray(getattr(w, "kshift", (0.0, 0.0, 0.0)), dtype=np.float64)
        s1, s2, s3 = self.kshift
        self.kfrac = np.array([((i1 + s1) / n1, (i2 + s2) / n2, (i3 + s3) / n3) for i1 in range(n1)
                               for i2 in range(n2) for i3 in range(n3)])
        # band (zero-weight) k-points off the mesh (Sec. 2.5, band-structure calculation): their
        # orbitals are targets of every term and partners of none; their fillings enter only the
        # divergence corrections.  k indices nk .. nk + nkb - 1.
        bk = getattr(w, "band_k", None)
        self.nkb = 0 if bk is None else len(bk)
        self.kall = self.kfrac if not self.nkb else np.concatenate(
            [self.kfrac, np.asarray(bk, dtype=np.float64).reshape(-1, 3)])
        self.grid = tuple(int(x) for x in w.grid)
        self.nr = int(np.prod(self.grid))
        self.alpha = float(w.alpha if alpha is None else alpha)
        self.div = bool(div_correction)
        if reading not in ("printed", "limit"):
            raise ValueError("reading must be 'printed' or 'limit'")
        self.reading = reading
        # u~_short(0)/N_k count in the G = G' = 0 corrections of 3a2 and 3b6 (reading R4)
        self.ushort_mult = 1.0 if reading == "printed" else 2.0
        self.A = torch.as_tensor(w.A if A is None else A, dtype=RD)
        self.C = torch.as_tensor(w.C if C is None else C, dtype=RD)
        ms = [np.fft.fftfreq(N, 1.0 / N).astype(np.int64) for N in self.grid]
        self.mgrid = np.stack(np.meshgrid(*ms, indexing="ij"), -1)            # (N1,N2,N3,3)
        nyq = np.zeros(self.grid, dtype=bool)
        for i, N in enumerate(self.grid):
            if N % 2 == 0:
                nyq |= self.mgrid[..., i] == -N // 2
        self.nyq = torch.as_tensor(nyq)
        self.negidx = [torch.as_tensor((-np.arange(N)) % N) for N in self.grid]
        self._kcache: Dict = {}
        # optional sample of target orbitals: terms are then evaluated for these targets only
        # (the other rows are returned as zeros); partner sums are untouched
        self.tsel = None
        # orbitals
        cr = [torch.as_tensor(c, dtype=CD) for c in w.right] if coeff is None else list(coeff)
        if left is not None:
            cl = list(left)
        elif w.left is not None:
            cl = [torch.as_tensor(c, dtype=CD) for c in w.left]
        else:
            cl = None
        if cl is not None and biorthogonalize:
            cr, cl = biorthogonalize_coeffs(cr, cl)
        self.cr, self.cl = cr, cl
        self.occ = [torch.as_tensor(o, dtype=RD) for o in w.occ]
        # spin channels (Sec. 2.1, Eq. SCF: one orbital set per spin; unpolarized input: the same set)
        self.polarized = getattr(w, "right_dn", None) is not None
        if self.polarized:
            crd = [torch.as_tensor(c, dtype=CD) for c in w.right_dn] if coeff_dn is None else list(coeff_dn)
            if left_dn is not None:
                cld = list(left_dn)
            else:
                cld = None if w.left_dn is None else [torch.as_tensor(c, dtype=CD) for c in w.left_dn]
            if cld is not None and biorthogonalize:
                crd, cld = biorthogonalize_coeffs(crd, cld)
            occd = [torch.as_tensor(o, dtype=RD) for o in (w.occ_dn if w.occ_dn is not None else w.occ)]
            self.spin_sets = [(cr, cl, self.occ), (crd, cld, occd)]
        else:
            self.spin_sets = [(cr, cl, self.occ)] * 2
        self.miller = [np.asarray(m, dtype=np.int64) for m in w.miller]
        if self.nkb:
            assert cl is None and not self.polarized, "band k-points are built for TC mode with one spin channel"
            self.miller += [np.asarray(m, dtype=np.int64) for m in w.band_miller]
        self._build_orbitals()
        self._gb()

    # ---------------------------------------------------------------- setup
    def FT(self, f):
        return torch.fft.fftn(f, dim=(-3, -2, -1)) / self.nr

    def IFT(self, F):
        return torch.fft.ifftn(F, dim=(-3, -2, -1)) * self.nr

    def neg(self, F):
        """F(-G) on the grid (index negation modulo N)."""
        i1, i2, i3 = self.negidx
        return F[..., i1, :, :][..., :, i2, :][..., :, :, i3]

    def _to_real(self, c, ik, grad=False):
        """Cell-periodic part (or (nabla + ik) of it) on the grid, Sec. 2.3."""
        N1, N2, N3 = self.grid
        m = self.miller[ik]
        nb = c.shape[0]
        if grad:
            kg = torch.as_tensor((self.kall[ik][None, :] + m) @ self.B, dtype=RD)  # (npw,3)
            out = []
            for a in range(3):
                box = torch.zeros((nb, N1, N2, N3), dtype=CD)
                box[:, m[:, 0] % N1, m[:, 1] % N2, m[:, 2] % N3] = c * (1j * kg[:, a])[None, :]
                out.append(self.IFT(box) / math.sqrt(self.omega))
            return torch.stack(out, 1)
        box = torch.zeros((nb, N1, N2, N3), dtype=CD)
        box[:, m[:, 0] % N1, m[:, 1] % N2, m[:, 2] % N3] = c
        return self.IFT(box) / math.sqrt(self.omega)

    def _channel(self, cr, cl, occ):
        phi, chi, D, kidx, f = [], [], [], [], []
        for ik in range(self.nk):
            p = self._to_real(cr[ik], ik)
            phi.append(p)
            chi.append(p if cl is None else self._to_real(cl[ik], ik))
            D.append(self._to_real(cr[ik], ik, grad=True))
            kidx += [ik] * p.shape[0]
            f.append(occ[ik])
        w = torch.cat(f) / self.nk
        for b in range(self.nkb):   # band orbitals: fillings for the corrections, zero partner weight
            ik = self.nk + b
            c = torch.as_tensor(self.w.band_right[b], dtype=CD)
            p = self._to_real(c, ik)
            phi.append(p)
            chi.append(p)
            D.append(self._to_real(c, ik, grad=True))
            kidx += [ik] * p.shape[0]
            f.append(torch.as_tensor(self.w.band_occ[b], dtype=RD))
        f = torch.cat(f)
        w = torch.cat([w, torch.zeros(f.shape[0] - w.shape[0], dtype=RD)])
        return dict(phi=torch.cat(phi), chi=torch.cat(chi), D=torch.cat(D), f=f, w=w,
                    k=np.array(kidx, dtype=np.int64))

    def _build_orbitals(self):
        # one orbital set per spin channel; unpolarized input: both channels hold the same orbitals
        up = self._channel(*self.spin_sets[0])
        self.orb = [up, self._channel(*self.spin_sets[1]) if self.polarized else up]
        self.P = up["phi"].shape[0]                      # targets: mesh and band orbitals
        self.Pm = int(np.sum(up["k"] < self.nk))           # partners: the mesh orbitals
        assert self.orb[1]["phi"].shape[0] == self.P, "the same number of bands per spin channel is assumed"
        self.n = [torch.sum(o["w"][:, None, None, None] * torch.conj(o["chi"]) * o["phi"], 0)
                  for o in self.orb]
        self.J = [torch.sum(o["w"][:, None, None, None, None] * torch.conj(o["chi"])[:, None] * o["D"], 0)
                  for o in self.orb]
        self.nG = [self.FT(x) for x in self.n]
        self.JG = [self.FT(x) for x in self.J]

    def qvec(self, delta):
        """Cartesian Q = Delta + G on the grid, Delta in fractional units of b."""
        return torch.as_tensor((np.asarray(delta)[None, None, None, :] + self.mgrid) @ self.B, dtype=RD)

    def kern(self, delta, mode, s):
        """Kernel tables at Q = Delta + G for channel s; mode 'H' (Hartree) or 'X' (exchange).

        Returns (Q (N..,3), V2a, u~) with the Q = 0 and Nyquist conventions R1, R2.
        """
        key = (tuple(np.round(np.asarray(delta, dtype=np.float64), 12)), mode, s)
        if key in self._kcache:
            return self._kcache[key]
        Q = self.qvec(delta)
        Q2 = torch.sum(Q * Q, -1)
        zero = Q2 < 1e-20
        Q2s = torch.where(zero, torch.ones_like(Q2), Q2)
        A, C = self.A[s], self.C[s]
        ut, lap, W = jastrow_kernels(Q2s, A, C)
        v = FOURPI / Q2s
        V = v + lap - W
        if mode == "H":
            V = torch.where(zero, torch.zeros_like(V), V)
        else:
            V0 = -FOURPI * A - 2.0 * math.pi * A * A / C          # v(0) := 0, L(0) - W(0)
            V = torch.where(zero, V0 * torch.ones_like(V), V)
        ut = torch.where(zero, torch.zeros_like(ut), ut)           # vector kernel iQu := 0 at Q = 0
        keep = ~self.nyq
        V = torch.where(keep, V, torch.zeros_like(V))
        ut = torch.where(keep, ut, torch.zeros_like(ut))
        Qt = Q.permute(3, 0, 1, 2).contiguous()                    # (3,N1,N2,N3)
        out = (Qt, V, ut)
        self._kcache[key] = out
        return out

    def _gb(self):
        """Gygi-Baldereschi constant of Eq. correction2 with A_aux = exp(-alpha q^2)/q^2.

        Sigma_aux = sum over the mesh q and all G (ball exp(-alpha|k-q+G|^2) > 1e-18) of
        A_aux(k-q+G), excluding k-q+G = 0; k and q both on the mesh, so k - q runs over the unshifted
        mesh whatever its shift, and k = 0 with the unshifted points is used.  Also
        returns the vector sum of Eq. correction_nabla (zero on a uniform mesh).
        """
        a = self.alpha
        qmax = math.sqrt(41.45 / a)
        lens = np.linalg.norm(self.lattice, axis=1)
        mmax = [int(math.ceil(qmax * L / (2 * math.pi))) + 2 for L in lens]
        rr = [np.arange(-m, m + 1) for m in mmax]
        M = np.stack(np.meshgrid(*rr, indexing="ij"), -1).reshape(-1, 3).astype(np.float64)
        tot = 0.0
        vec = np.zeros(3)
        for q in self.kfrac - (self.kshift / np.asarray(self.kmesh, dtype=np.float64))[None, :]:
            Q = (M - q[None, :]) @ self.B
            q2 = np.sum(Q * Q, 1)
            ok = (q2 > 1e-20) & (a * q2 < 41.45)
            t = np.exp(-a * q2[ok]) / q2[ok]
            tot += math.fsum(t)
            vec += (Q[ok] * t[:, None]).sum(0)
        self.sigma_aux = tot
        self.gb_vector = vec / self.nk
        self.delta_gb = self.omega / (4.0 * math.sqrt(math.pi ** 3 * a)) - (-a + tot) / self.nk

    def is_band(self, j):
        return self.orb[0]["k"][j] >= self.nk

    def band_set(self, s, j):
        """Band target j: its k-point's orbitals (q_k of the band forms), the GB quantities there and
        4 pi A_par (the parallel channel of the exchange-type terms)."""
        ik = self.orb[s]["k"][j]
        dgb, V = self.gb_band(ik)
        return self.sel(s, ik), dgb, torch.as_tensor(V, dtype=RD), FOURPI * self.A[0]

    def vdot(self, V, X):
        """V . X over the leading vector axis of X (V Cartesian, real)."""
        return sum(V[c] * X[c] for c in range(3))

    def gb_band(self, ik):
        """GB quantities at a band k-point (off the mesh, so no k - q + G vanishes): the bracket of
        Eq. correction with the mesh sum S = sum_{q,G} A_aux(k - q + G), divided by 4 pi as delta_gb is,
        and the vector sum of Eq. correction_nabla taken at the same arguments (reading R13),
        V = sum_{q,G} (k - q + G) A_aux(k - q + G) (Cartesian).  Returns (delta_gb_band, V / N_k)."""
        key = ("gb_band", ik)
        if key in self._kcache:
            return self._kcache[key]
        a = self.alpha
        qmax = math.sqrt(41.45 / a)
        lens = np.linalg.norm(self.lattice, axis=1)
        mmax = [int(math.ceil(qmax * L / (2 * math.pi))) + 3 for L in lens]
        rr = [np.arange(-m, m + 1) for m in mmax]
        M = np.stack(np.meshgrid(*rr, indexing="ij"), -1).reshape(-1, 3).astype(np.float64)
        tot, vec = 0.0, np.zeros(3)
        for q in self.kfrac:
            Q = (M + (self.kall[ik] - q)[None, :]) @ self.B
            q2 = np.sum(Q * Q, 1)
            ok = a * q2 < 41.45
            t = np.exp(-a * q2[ok]) / q2[ok]
            tot += math.fsum(t)
            vec += (Q[ok] * t[:, None]).sum(0)
        out = (self.omega / (4.0 * math.sqrt(math.pi ** 3 * a)) - tot / self.nk, vec / self.nk)
        self._kcache[key] = out
        return out

    # ---------------------------------------------------------------- helpers
    def sel(self, s, ik=None):
        o = self.orb[s]
        if ik is None:
            return np.arange(self.P)
        return np.nonzero(o["k"] == ik)[0]

    def restrict_targets(self, targets):
        """Evaluate the operator only on the given target orbitals (sampled checks at full size)."""
        self.tsel = None if targets is None else np.unique(np.asarray(targets, dtype=np.int64))

    def sel_t(self, s, ik):
        """Targets at k-point ik (all orbitals of ik unless a target sample is set)."""
        J = self.sel(s, ik)
        return J if self.tsel is None else J[np.isin(J, self.tsel)]

    def is_target(self, j):
        return self.tsel is None or bool(np.isin(j, self.tsel))

    def rho0(self, a, b):
        """FT[chi_a^* phi_b](0) = <chi_a|phi_b>/Omega (periodic parts)."""
        return torch.mean(a * b, dim=(-3, -2, -1))

    def conv(self, delta, mode, s, F, kind):
        """Apply a kernel to G-space data F: 'V' scalar V2a, 'U' vector iQu, 'Ud' -iQu . (vector F)."""
        Q, V, ut = self.kern(delta, mode, s)
        if kind == "V":
            return self.IFT(V * F)
        if kind == "U":
            return self.IFT(1j * Q * ut * F.unsqueeze(-4))
        if kind == "Ud":
            return self.IFT(torch.sum(-1j * Q * ut * F, -4))
        raise ValueError(kind)

    def dk(self, kt, kq):
        return self.kall[kt] - self.kall[kq]

    # ---------------------------------------------------------------- two-body
    def t_2ah(self, s):
        """Alg. 2ah: sum_s' V2a^{s s'} n~_s' (G != 0) back-transformed, times phi_j."""
        h = sum(self.conv(np.zeros(3), "H", _pair(s, s2), self.nG[s2], "V") for s2 in range(2))
        return h[None] * self.orb[s]["phi"]

    def t_2bh1(self, s):
        """2bh1 'in the same way as' Alg. 2ah: [sum_s' iGu~ n~_s'] . (nabla+ik) phi_j."""
        h = sum(self.conv(np.zeros(3), "H", _pair(s, s2), self.nG[s2], "U") for s2 in range(2))
        return torch.sum(h[None] * self.orb[s]["D"], 1)

    def t_2bh2(self, s):
        """2bh2: -[sum_s' iGu~ . J~_s'] phi_j with J = sum_q w chi_q^* (nabla+ik) phi_q (grad_2 u_12 = -grad u)."""
        h = sum(self.conv(np.zeros(3), "H", _pair(s, s2), self.JG[s2], "Ud") for s2 in range(2))
        return h[None] * self.orb[s]["phi"]

    def _exchange_loop(self, s, body):
        o = self.orb[s]
        acc = {}
        for q in range(self.Pm):
            for kt in range(self.nk + self.nkb):
                J = self.sel_t(s, kt)
                if len(J) == 0:
                    continue
                d = self.dk(kt, o["k"][q])
                contrib = body(q, J, d)
                for jj, j in enumerate(J):
                    acc[j] = acc.get(j, 0) + contrib[jj]
        zero = torch.zeros_like(o["phi"][0])
        return torch.stack([acc.get(j, zero) for j in range(self.P)])

    def t_2ax(self, s):
        """Alg. 2ax (+ Eq. divcorr_2ax_scf)."""
        o = self.orb[s]

        def body(q, J, d):
            rho = torch.conj(o["chi"][q])[None] * o["phi"][J]
            h2 = self.conv(d, "X", 0, self.FT(rho), "V")
            return -h2 * o["phi"][q][None] * o["w"][q]
        g = self._exchange_loop(s, body)
        if self.div:
            g = g + self.c_2ax(s)
        return g

    def c_2ax(self, s):
        """Eq. divcorr_2ax_scf: -4 pi Delta_GB sum_mu f rho~_{(k mu), j}(0) phi_{k mu}."""
        o = self.orb[s]
        out = []
        for j in range(self.P):
            if not self.is_target(j):
                out.append(torch.zeros_like(o["phi"][0]))
                continue
            Q = self.sel(s, o["k"][j])
            r0 = self.rho0(torch.conj(o["chi"][Q]), o["phi"][j][None])   # (nb,)
            # band k-point: Eq. divcorr_2ax_band (no excluded term and no alpha)
            dgb = self.delta_gb if o["k"][j] < self.nk else self.gb_band(o["k"][j])[0]
            out.append(-FOURPI * dgb * torch.sum((o["f"][Q] * r0)[:, None, None, None] * o["phi"][Q], 0))
        return torch.stack(out)

    def t_2bx1(self, s):
        """2bx1 'in the same way as' Alg. 2ax: -sum_q w [iQu~ (*) chi_q^* phi_j] . (nabla+ik_q) phi_q."""
        o = self.orb[s]

        def body(q, J, d):
            rho = torch.conj(o["chi"][q])[None] * o["phi"][J]
            h = self.conv(d, "X", 0, self.FT(rho), "U")
            return -torch.sum(h * o["D"][q][None], 1) * o["w"][q]
        g = self._exchange_loop(s, body)
        if self.div and self.nkb:
            g = g + self._band_corr(s, self.c_2bx1_band)
        if self.div and self.reading == "limit":
            g = g + self.c_2bx1_mesh(s)
        return g

    def c_2bx1_mesh(self, s):
        """Reading R4 "limit": the remainder -(4 pi A_par / N_k) sum_mu f rho~_{mu j}(0) phi_mu of a mesh
        target j (the band operator's limit at a mesh point; zero rows for band targets)."""
        o = self.orb[s]
        out = []
        for j in range(self.P):
            if not self.is_target(j) or self.is_band(j):
                out.append(torch.zeros_like(o["phi"][0]))
                continue
            Q = self.sel(s, o["k"][j])
            r0 = self.rho0(torch.conj(o["chi"][Q]), o["phi"][j][None])
            out.append(-FOURPI * self.A[0] / self.nk
                       * torch.sum((o["f"][Q] * r0)[:, None, None, None] * o["phi"][Q], 0))
        return torch.stack(out)

    def _band_corr(self, s, fn):
        """Stack fn(s, j) over the band targets (zeros elsewhere)."""
        o = self.orb[s]
        zero = torch.zeros_like(o["phi"][0])
        return torch.stack([fn(s, j) if (self.is_band(j) and self.is_target(j)) else zero for j in range(self.P)])

    def c_2bx1_band(self, s, j):
        """Eq. divcorr_2bx1 (band k): i 4 pi A V . sum_mu f rho~_{mu j}(0) (nabla + ik) phi_mu."""
        o = self.orb[s]
        Q, _, V, a4 = self.band_set(s, j)
        r0 = self.rho0(torch.conj(o["chi"][Q]), o["phi"][j][None])
        DV = sum(V[c] * o["D"][Q][:, c] for c in range(3))
        return 1j * a4 * torch.sum((o["f"][Q] * r0)[:, None, None, None] * DV, 0)

    def t_2bx2(self, s):
        """2bx2: +sum_q w [iQu~ . (*) chi_q^* (nabla+ik) phi_j] phi_q (grad_2 u_21 = -grad_1 u_12)."""
        o = self.orb[s]

        def body(q, J, d):
            rho = torch.conj(o["chi"][q])[None, None] * o["D"][J]
            h = -self.conv(d, "X", 0, self.FT(rho), "Ud")
            return h * o["phi"][q][None] * o["w"][q]
        g = self._exchange_loop(s, body)
        if self.div and self.nkb:
            g = g + self._band_corr(s, self.c_2bx2_band)
        return g

    def c_2bx2_band(self, s, j):
        """Eq. divcorr_2bx2 (band k): -i 4 pi A sum_mu f (V . FT[chi_mu^* (nabla+ik) phi_j](0)) phi_mu."""
        o = self.orb[s]
        Q, _, V, a4 = self.band_set(s, j)
        x = torch.mean(torch.conj(o["chi"][Q])[:, None] * o["D"][j][None], dim=(-3, -2, -1))   # (nq, 3)
        c = torch.sum(x * V[None, :], 1)
        return -1j * a4 * torch.sum((o["f"][Q] * c)[:, None, None, None] * o["phi"][Q], 0)

    # ---------------------------------------------------------------- three-body
    def h1(self, s):
        """h1^s = FT^-1[sum_s2 iG u~^{s s2} n~_s2] (Algs. 3a1, 3a3, 3b1, 3b3)."""
        return sum(self.conv(np.zeros(3), "H", _pair(s, s2), self.nG[s2], "U") for s2 in range(2))

    def t_3a1(self, s):
        """Alg. 3a1 with the bilinear h1 . h1 (reading R6)."""
        h1 = self.h1(s)
        return -0.5 * torch.sum(h1 * h1, 0)[None] * self.orb[s]["phi"]

    def h5_3a2(self, s, q2, s2):
        """h5^{s,s2}(r; q2) of Alg. 3a2 for occupied q2 of spin s2 (+ its corrections)."""
        o2 = self.orb[s2]
        ch = _pair(s, s2)
        h5 = 0
        for q1 in range(self.Pm):
            d21 = self.kall[o2["k"][q1]] - self.kall[o2["k"][q2]]
            h2 = self.conv(d21, "X", ch, self.FT(torch.conj(o2["chi"][q2]) * o2["phi"][q1]), "U")
            h4 = self.conv(-d21, "X", ch, self.FT(torch.conj(o2["chi"][q1]) * o2["phi"][q2]), "U")
            h5 = h5 + torch.sum(h2 * h4, 0) * o2["w"][q1]
        if self.div:
            h5 = h5 + self.c_3a2(ch, q2, s2)
        return h5

    def c_3a2(self, ch, q2, s2):
        """Corrections to h5 (Eqs. divcor_3a2_first/second, general-overlap form)."""
        o2 = self.orb[s2]
        A, C = self.A[ch], self.C[ch]
        ushort = -FOURPI * A * C * C                                   # Eq. u_short
        c1 = FOURPI * A * (FOURPI * A * self.delta_gb + self.ushort_mult * ushort / self.nk)   # R4
        _, _, utH = self.kern(np.zeros(3), "H", ch)
        out = 0
        for q1 in self.sel(s2, o2["k"][q2]):
            r21 = self.FT(torch.conj(o2["chi"][q2]) * o2["phi"][q1])
            r12 = self.FT(torch.conj(o2["chi"][q1]) * o2["phi"][q2])
            f1 = o2["f"][q1]
            out = out + c1 * f1 * r21[0, 0, 0] * r12[0, 0, 0]
            F = utH * (r21 * r12[0, 0, 0] + r21[0, 0, 0] * r12)
            out = out + FOURPI * A / self.nk * f1 * self.IFT(F)
        return out

    def t_3a2(self, s):
        """Alg. 3a2: g_j = h6 phi_j / 2 with h6 = sum_s2 sum_q2 w_q2 h5^{s,s2}(q2)."""
        h6 = 0
        for s2 in range(2):
            for q2 in range(self.Pm):
                h6 = h6 + self.h5_3a2(s, q2, s2) * self.orb[s2]["w"][q2]
        return 0.5 * h6[None] * self.orb[s]["phi"]

    def h4_3a3(self, s, j):
        """h4 of Alg. 3a3 for target j (equals h3 of Alg. 3b4, reading R5)."""
        o = self.orb[s]
        h4 = 0
        for q1 in range(self.Pm):
            d = self.dk(o["k"][j], o["k"][q1])
            h3 = self.conv(d, "X", 0, self.FT(torch.conj(o["chi"][q1]) * o["phi"][j]), "U")
            h4 = h4 + h3 * o["phi"][q1][None] * o["w"][q1]
        if self.div and self.is_band(j):
            # Eq. divcorr_3a3 (= Eq. div_corr_3b4_2): -i 4 pi A V sum_mu f rho~_{mu j}(0) phi_mu
            Q, _, V, a4 = self.band_set(s, j)
            r0 = self.rho0(torch.conj(o["chi"][Q]), o["phi"][j][None])
            p = torch.sum((o["f"][Q] * r0)[:, None, None, None] * o["phi"][Q], 0)
            h4 = h4 + (-1j * a4) * V[:, None, None, None] * p[None]
        return h4

    def t_3a3(self, s):
        """Alg. 3a3: g_j = h1 . h4 / 2."""
        h1 = self.h1(s)
        zero = torch.zeros_like(self.orb[s]["phi"][0])
        return torch.stack([0.5 * torch.sum(h1 * self.h4_3a3(s, j), 0) if self.is_target(j) else zero
                            for j in range(self.P)])

    def h3_3a4(self, s, q2):
        """h3^{s2}(r; q2) of Alg. 3a4 (q2 of spin s, same-spin partners q1)."""
        o = self.orb[s]
        h3 = 0
        for q1 in range(self.Pm):
            d = self.kall[o["k"][q2]] - self.kall[o["k"][q1]]
            h2 = self.conv(d, "X", 0, self.FT(torch.conj(o["chi"][q1]) * o["phi"][q2]), "U")
            h3 = h3 + h2 * o["phi"][q1][None] * o["w"][q1]
        return h3

    def t_3a4(self, s):
        """Alg. 3a4: g_j = -1/2 sum_q2 w_q2 h3(q2) . [iQu~ (*) chi_q2^* phi_j]."""
        o = self.orb[s]
        g = torch.zeros_like(o["phi"])
        for q2 in range(self.Pm):
            h3 = self.h3_3a4(s, q2)
            for kt in range(self.nk + self.nkb):
                J = self.sel_t(s, kt)
                if len(J) == 0:
                    continue
                d = self.dk(kt, o["k"][q2])
                h5 = self.conv(d, "X", 0, self.FT(torch.conj(o["chi"][q2])[None] * o["phi"][J]), "U")
                g[J] = g[J] - 0.5 * torch.sum(h3[None] * h5, 1) * o["w"][q2]
        if self.div and self.nkb:
            def corr(s_, j):
                # the q2 sum of the algorithm at q2 -> k (Eq. div_corr_3a4_2) and the q1 sum inside h3 of
                # the band orbitals (Eq. div_corr_3a4_3), with the algorithm's i^2 = -1 kept (reading R14):
                #   +(i/2) 4 pi A sum_mu2 f rho~_{mu2 j}(0) V . h3(mu2)
                #   +(1/2) (4 pi A)^2 V.V sum_{mu1 mu2} f f rho~_{mu1 mu2}(0) rho~_{mu2 j}(0) phi_mu1
                Q, _, V, a4 = self.band_set(s_, j)
                f = o["f"][Q]
                r0 = self.rho0(torch.conj(o["chi"][Q]), o["phi"][j][None])                    # (nq,)
                out = 0
                for i2, m2 in enumerate(Q):
                    out = out + 0.5j * a4 * f[i2] * r0[i2] * self.vdot(V, self.h3_3a4(s_, m2))
                S = self.rho0(torch.conj(o["chi"][Q])[:, None], o["phi"][Q][None])              # (nq, nq)
                cvec = (S * (f * r0)[None, :]).sum(1) * f                                         # over mu2
                out = out + 0.5 * a4 * a4 * float(V @ V) * torch.sum(cvec[:, None, None, None] * o["phi"][Q], 0)
                return out
            g = g + self._band_corr(s, corr)
        return g

    def t_3b1(self, s):
        """Alg. 3b1."""
        h3 = 0
        for s1 in range(2):
            h2 = self.h1(s1) * self.n[s1][None]
            h3 = h3 + self.conv(np.zeros(3), "H", _pair(s, s1), self.FT(h2), "Ud")
        return -0.5 * h3[None] * self.orb[s]["phi"]

    def h3_3b2(self, s2, q2):
        """h3^{s2}(r; q2) of Algs. 3b2 / 3b5."""
        o = self.orb[s2]
        h3 = 0
        for q1 in range(self.Pm):
            d = self.kall[o["k"][q1]] - self.kall[o["k"][q2]]
            h2 = self.conv(d, "X", 0, self.FT(torch.conj(o["chi"][q2]) * o["phi"][q1]), "U")
            h3 = h3 + h2 * torch.conj(o["chi"][q1])[None] * o["w"][q1]
        return h3

    def t_3b2(self, s):
        """Alg. 3b2."""
        h6 = 0
        for s2 in range(2):
            o2 = self.orb[s2]
            h5 = 0
            for q2 in range(self.Pm):
                h5 = h5 + self.h3_3b2(s2, q2) * o2["phi"][q2][None] * o2["w"][q2]
            h6 = h6 + self.conv(np.zeros(3), "H", _pair(s, s2), self.FT(h5), "Ud")
        return 0.5 * h6[None] * self.orb[s]["phi"]

    def t_3b3(self, s):
        """Alg. 3b3."""
        o = self.orb[s]
        h1 = self.h1(s)

        def body(q, J, d):
            h2 = h1[None] * (torch.conj(o["chi"][q])[None] * o["phi"][J])[:, None]
            h3 = self.conv(d, "X", 0, self.FT(h2), "Ud")
            return 0.5 * h3 * o["phi"][q][None] * o["w"][q]
        g = self._exchange_loop(s, body)
        if self.div and self.nkb:
            def corr(s_, j):
                # Eq. div_corr_3b3_2: (i/2) 4 pi A sum_mu f (V . FT[chi_mu^* phi_j h1](0)) phi_mu
                Q, _, V, a4 = self.band_set(s_, j)
                x = torch.mean(torch.conj(o["chi"][Q])[:, None] * (o["phi"][j][None] * h1)[None],
                               dim=(-3, -2, -1))
                c = torch.sum(x * V[None, :], 1)
                return 0.5j * a4 * torch.sum((o["f"][Q] * c)[:, None, None, None] * o["phi"][Q], 0)
            g = g + self._band_corr(s, corr)
        return g

    def t_3b4(self, s):
        """Alg. 3b4 (with reading R5)."""
        o = self.orb[s]
        g = []
        for j in range(self.P):
            if not self.is_target(j):
                g.append(torch.zeros_like(o["phi"][0]))
                continue
            h3 = self.h4_3a3(s, j)
            acc = 0
            for q1 in range(self.Pm):
                d = self.dk(o["k"][j], o["k"][q1])
                h4 = h3 * torch.conj(o["chi"][q1])[None]
                h5 = self.conv(d, "X", 0, self.FT(h4), "Ud")
                acc = acc - 0.5 * h5 * o["phi"][q1] * o["w"][q1]
            if self.div and self.is_band(j):
                # Eq. div_corr_3b4_4: -(i/2) 4 pi A sum_mu f (V . FT[chi_mu^* h3](0)) phi_mu
                Q, _, V, a4 = self.band_set(s, j)
                x = torch.mean(torch.conj(o["chi"][Q])[:, None] * h3[None], dim=(-3, -2, -1))   # (nq, 3)
                c = torch.sum(x * V[None, :], 1)
                acc = acc - 0.5j * a4 * torch.sum((o["f"][Q] * c)[:, None, None, None] * o["phi"][Q], 0)
            g.append(acc)
        return torch.stack(g)

    def t_3b5(self, s):
        """Alg. 3b5 with the sign of its caption, the term list and Eq. 3b5_div (reading R9)."""
        o = self.orb[s]
        g = torch.zeros_like(o["phi"])
        for q2 in range(self.Pm):
            h3 = self.h3_3b2(s, q2)
            for kt in range(self.nk + self.nkb):
                J = self.sel_t(s, kt)
                if len(J) == 0:
                    continue
                d = self.dk(kt, o["k"][q2])
                h4 = h3[None] * o["phi"][J][:, None]
                h5 = self.conv(d, "X", 0, self.FT(h4), "Ud")
                g[J] = g[J] - 0.5 * h5 * o["phi"][q2][None] * o["w"][q2]
        if self.div and self.nkb:
            def corr(s_, j):
                # the q2 sum at q2 -> k (Eq. 3b5_div_2) and the q1 sum inside h3 of the band orbitals
                # (Eq. 3b5_div_3), signs from the algorithm (reading R14):
                #   -(i/2) 4 pi A sum_mu2 f (V . FT[h3(mu2) phi_j](0)) phi_mu2
                #   +(1/2) (4 pi A)^2 V.V sum_{mu1 mu2} f f rho~_{mu2 mu1}(0) rho~_{mu1 j}(0) phi_mu2
                Q, _, V, a4 = self.band_set(s_, j)
                f = o["f"][Q]
                out = 0
                for i2, m2 in enumerate(Q):
                    x = torch.mean(self.h3_3b2(s_, m2) * o["phi"][j][None], dim=(-3, -2, -1))   # (3,)
                    out = out - 0.5j * a4 * f[i2] * torch.sum(x * V) * o["phi"][m2]
                S = self.rho0(torch.conj(o["chi"][Q])[:, None], o["phi"][Q][None])              # S[mu2, mu1]
                r0 = self.rho0(torch.conj(o["chi"][Q]), o["phi"][j][None])                    # rho~_{mu1 j}
                cvec = (S * (f * r0)[None, :]).sum(1) * f                                         # per mu2
                out = out + 0.5 * a4 * a4 * float(V @ V) * torch.sum(cvec[:, None, None, None] * o["phi"][Q], 0)
                return out
            g = g + self._band_corr(s, corr)
        return g

    def t_3b6(self, s):
        """Alg. 3b6 (+ Eqs. 3b6_div_scf1-3)."""
        o = self.orb[s]

        def body(q, J, d):
            h1 = self.FT(torch.conj(o["chi"][q])[None] * o["phi"][J])
            h4 = 0
            for s1 in range(2):
                ch = _pair(s1, s)
                h2 = self.conv(d, "X", ch, h1, "U")
                h3 = h2 * self.n[s1][None, None]
                h4 = h4 + self.conv(d, "X", ch, self.FT(h3), "Ud")
            return 0.5 * h4 * o["phi"][q][None] * o["w"][q]
        g = self._exchange_loop(s, body)
        if self.div:
            g = g + self.c_3b6(s)
        return g

    def c_3b6(self, s):
        """Eqs. 3b6_div_scf1, 3b6_div_scf2, 3b6_div_scf3 (index typos read as u^{s1 s})."""
        o = self.orb[s]
        out = []
        for j in range(self.P):
            if not self.is_target(j):
                out.append(torch.zeros_like(o["phi"][0]))
                continue
            Q = self.sel(s, o["k"][j])
            acc = 0
            band = self.is_band(j)
            if band:
                dgb_b, V = self.gb_band(o["k"][j])
                V = torch.as_tensor(V, dtype=RD)
                Gc = self.qvec(np.zeros(3))                                     # Cartesian G (N1,N2,N3,3)
                VG = torch.sum(Gc * V, -1)
            for s1 in range(2):
                ch = _pair(s1, s)
                A, C = self.A[ch], self.C[ch]
                _, _, utH = self.kern(np.zeros(3), "H", ch)
                nG = self.nG[s1]
                if not band:
                    ushort = -FOURPI * A * C * C
                    c1 = 2.0 * math.pi * A * (FOURPI * A * self.delta_gb
                                              + self.ushort_mult * ushort / self.nk)   # R4
                    field = self.IFT(utH * nG)
                else:
                    # Eqs. 3b6_div_band1-3: band GB bracket without alpha and u_short; the G' != 0 and
                    # G + G' = 0 parts through the vector sum of Eq. correction_nabla
                    c1 = 2.0 * math.pi * A * FOURPI * A * dgb_b
                    field = -2.0 * math.pi * A * self.IFT(VG * utH * nG)
                for q2 in Q:
                    rG = self.FT(torch.conj(o["chi"][q2]) * o["phi"][j])
                    r0 = rG[0, 0, 0]
                    t1 = c1 * r0 * nG[0, 0, 0]
                    if not band:
                        t3 = 2.0 * math.pi * A / self.nk * torch.sum(utH * rG * self.neg(nG))
                        t2 = 2.0 * math.pi * A / self.nk * r0 * field
                    else:
                        t3 = -2.0 * math.pi * A * torch.sum(VG * utH * rG * self.neg(nG))
                        t2 = r0 * field
                    acc = acc + o["f"][q2] * (t1 + t3 + t2) * o["phi"][q2]
            out.append(acc)
        return torch.stack(out)

    # ---------------------------------------------------------------- assembly
    def term(self, name, s):
        return getattr(self, "t_" + name)(s)

    def apply_terms(self, terms=ALL_TERMS, spins=(0, 1)):
        """{term: [g for each spin]} with the printed (unmultiplied) terms."""
        return {t: {s: self.term(t, s) for s in spins} for t in terms}

    def operator(self, terms=ALL_TERMS, s=0):
        """Two- and three-body operator on every orbital of spin s, split (h2 g, h3 g)."""
        g2 = 0
        g3 = 0
        for t in terms:
            g = self.term(t, s)
            if t in TERMS2:
                g2 = g2 + g
            else:
                g3 = g3 + MULT[t] * g
        return g2, g3

    def braket(self, s, g):
        """<chi_p | g_p> over the cell for every orbital p of spin s."""
        o = self.orb[s]
        return self.omega * torch.mean(torch.conj(o["chi"]) * g, dim=(-3, -2, -1))

    def kinetic(self, s=0):
        """<chi_p| -nabla^2/2 |phi_p> from the coefficients of spin channel s (Sec. 2.6.2)."""
        cr, clx, _ = self.spin_sets[s]
        out = []
        for ik in range(self.nk):
            kg = (self.kfrac[ik][None, :] + self.miller[ik]) @ self.B
            t = torch.as_tensor(0.5 * np.sum(kg * kg, 1), dtype=RD)
            cl = cr[ik] if clx is None else clx[ik]
            out.append(torch.sum(torch.conj(cl) * t[None, :] * cr[ik], 1))
        return torch.cat(out)

    def energy(self, terms=ALL_TERMS, with_kinetic=True, per_term=False):
        """Pseudo-energy per cell (reading R8), summed over both spin channels."""
        parts = {}
        for s in range(2):
            f = self.orb[s]["f"][:self.Pm]   # mesh orbitals only (band orbitals carry no weight)
            if with_kinetic:
                parts["T"] = parts.get("T", 0) + torch.sum(f * self.kinetic(s)).real / self.nk
            for t in terms:
                fac = 0.5 if t in TERMS2 else MULT[t] / 3.0
                e = torch.sum(f * self.braket(s, self.term(t, s))[:self.Pm]).real * fac / self.nk
                parts[t] = parts.get(t, 0) + e
        tot = sum(parts.values())
        return (tot, parts) if per_term else tot

    def to_coeff(self, g, s=0):
        """(Hc)(G) = sqrt(Omega) FT[g](G) on each orbital's plane-wave set."""
        o = self.orb[s]
        out = []
        for ik in range(self.nk + self.nkb):
            J = self.sel(s, ik)
            m = self.miller[ik]
            N1, N2, N3 = self.grid
            G = self.FT(g[J]) * math.sqrt(self.omega)
            out.append(G[:, m[:, 0] % N1, m[:, 1] % N2, m[:, 2] % N3])
        return out


def biorthogonalize_coeffs(cr, cl):
    """Normalize each right orbital, then make the left ones biorthogonal, <chi_i|phi_j> = delta_ij.

    Sec. 2.3 (BITC): left and right determinants with <chi_i|phi_j> = delta and <phi_i|phi_i> = 1.
    The left set is replaced by conj(S^-1) chi with S_ij = <chi_i|phi_j> (per k point).
    """
    rr, ll = [], []
    for r, l in zip(cr, cl):
        r = r / torch.linalg.norm(r, dim=1, keepdim=True)
        S = torch.conj(l) @ r.T
        l2 = torch.conj(torch.linalg.inv(S)) @ l
        rr.append(r)
        ll.append(l2)
    return rr, ll
