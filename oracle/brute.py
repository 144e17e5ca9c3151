"""Oracle O2: literal real-space integrals on tiny grids.

TEST INFRASTRUCTURE ONLY.  NumPy float64/complex128, no FFT.  Every two- and
three-body term is evaluated from its definition in Sec. 2.6 as an integral
over the full Bloch orbitals,

    <*, q1, q2 | O | a, b, c> = int dr2 dr3 chi*_q1(r2) chi*_q2(r3) O phi_a(r1) phi_b(r2) phi_c(r3),

with every permutation of the determinant (Eq. SCF / BITCSCF) taken separately
(3a1..3a6, 3b1..3b6, 3c1..3c6).  Orbitals are explicit plane-wave sums,
phi_p(r) = e^{ik.r} N_k^{-1/2} Omega^{-1/2} sum_G c(G) e^{iG.r}, and a
convolution with a kernel whose transform is K(Q) acts on a source of crystal
momentum Delta through the explicit matrix

    M[r1, r2] = (1/N_r) sum_{G in box} K(Delta + G) e^{i(Delta+G).(r1 - r2)},

which is the cell-grid quadrature of int dr2 K(r1 - r2) F(r2) for a
band-limited kernel (Eq. convolution).  The kernel conventions at Q = 0 and on
the Nyquist planes are those of the FFT-route oracle (its readings R1, R2);
divergence corrections are not part of this oracle.  The point of this module
is to check the factorised algorithms, their signs, the spin rules and the
multiplicities 3a5 = 3a4, 3a6 = 3a3, 3c* = 3b* against the definitions.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import torch

from .fftroute import jastrow_kernels

FOURPI = 4.0 * math.pi

# (name, sign, permutation of (j, q1, q2) into kets at (x1, x2, x3)); the sign
# is the determinant sign times the overall -1/2 of Eq. SCF, as listed in Sec. 2.6.4.
PERMS = [
    ("1", -0.5, (0, 1, 2)),
    ("2", +0.5, (0, 2, 1)),
    ("3", +0.5, (1, 0, 2)),
    ("4", -0.5, (1, 2, 0)),
    ("5", -0.5, (2, 0, 1)),
    ("6", +0.5, (2, 1, 0)),
]


def _pair(s1, s2):
    return 0 if s1 == s2 else 1


class Brute:
    def __init__(self, w, coeff=None, left=None, A=None, C=None):
        self.w = w
        lat = np.asarray(w.lattice, dtype=np.float64)
        self.omega = abs(float(np.linalg.det(lat)))
        self.B = 2.0 * math.pi * np.linalg.inv(lat).T
        n1, n2, n3 = w.kmesh
        self.nk = n1 * n2 * n3
        s1, s2, s3 = (float(x) for x in getattr(w, "kshift", (0.0, 0.0, 0.0)))   # Monkhorst-Pack shift
        self.kfrac = np.array([((i1 + s1) / n1, (i2 + s2) / n2, (i3 + s3) / n3) for i1 in range(n1)
                               for i2 in range(n2) for i3 in range(n3)])
        self.grid = tuple(w.grid)
        N1, N2, N3 = self.grid
        self.nr = N1 * N2 * N3
        idx = np.stack(np.meshgrid(np.arange(N1), np.arange(N2), np.arange(N3), indexing="ij"), -1).reshape(-1, 3)
        self.rfrac = idx / np.array(self.grid)[None, :]
        self.r = self.rfrac @ lat                                   # (Nr,3) cartesian
        ms = [np.fft.fftfreq(N, 1.0 / N).astype(np.int64) for N in self.grid]
        M = np.stack(np.meshgrid(*ms, indexing="ij"), -1).reshape(-1, 3)
        nyq = np.zeros(M.shape[0], dtype=bool)
        for i, N in enumerate(self.grid):
            if N % 2 == 0:
                nyq |= M[:, i] == -N // 2
        self.mbox = M
        self.nyqbox = nyq
        self.A = np.asarray(w.A if A is None else A, dtype=np.float64)
        self.C = np.asarray(w.C if C is None else C, dtype=np.float64)
        cr = [np.asarray(c) for c in (w.right if coeff is None else coeff)]
        cl = None
        if left is not None:
            cl = [np.asarray(c) for c in left]
        elif w.left is not None:
            cl = [np.asarray(c) for c in w.left]
        # full Bloch orbitals on the cell grid, spin list (unpolarized: the same orbitals in both channels;
        # polarized input: the down channel's own set, used as given)
        sets = [(cr, cl, w.occ)]
        if getattr(w, "right_dn", None) is not None:
            sets.append(([np.asarray(c) for c in w.right_dn],
                         None if w.left_dn is None else [np.asarray(c) for c in w.left_dn],
                         w.occ_dn if w.occ_dn is not None else w.occ))
        else:
            sets.append(sets[0])
        self.orbs = []
        for s, (crs, cls, occs) in enumerate(sets):
            for ik in range(self.nk):
                kg = (self.kfrac[ik][None, :] + w.miller[ik]) @ self.B     # (npw,3)
                E = np.exp(1j * self.r @ kg.T) / math.sqrt(self.nk * self.omega)  # (Nr,npw)
                for b in range(crs[ik].shape[0]):
                    self.orbs.append(dict(phi=E @ crs[ik][b], chi=E @ (crs[ik][b] if cls is None else cls[ik][b]),
                                          grad=np.stack([E @ (1j * kg[:, a] * crs[ik][b]) for a in range(3)]),
                                          k=ik, f=float(occs[ik][b]), s=s))
        self._mat = {}

    # ------------------------------------------------------------------ kernels
    def _tables(self, delta, ch, mode):
        Q = (np.asarray(delta)[None, :] + self.mbox) @ self.B
        Q2 = np.sum(Q * Q, 1)
        zero = Q2 < 1e-20
        Q2s = np.where(zero, 1.0, Q2)
        ut, lap, W = [x.numpy() for x in jastrow_kernels(torch.as_tensor(Q2s), torch.tensor(self.A[ch]),
                                                          torch.tensor(self.C[ch]))]
        V = FOURPI / Q2s + lap - W
        if mode == "H":
            V = np.where(zero, 0.0, V)
        else:
            V = np.where(zero, -FOURPI * self.A[ch] - 2 * math.pi * self.A[ch] ** 2 / self.C[ch], V)
        ut = np.where(zero, 0.0, ut)
        V = np.where(self.nyqbox, 0.0, V)
        ut = np.where(self.nyqbox, 0.0, ut)
        return Q, V, ut

    def mat(self, delta, ch, kind, mode="X"):
        """Convolution matrix for a source of crystal momentum delta (fractional)."""
        key = (tuple(np.round(delta, 12)), ch, kind, mode)
        if key in self._mat:
            return self._mat[key]
        Q, V, ut = self._tables(delta, ch, mode)
        E = np.exp(1j * self.r @ Q.T)                    # e^{i(Delta+G).r}
        if kind == "V":
            out = (E * V[None, :]) @ E.conj().T / self.nr
        else:                                            # vector kernel iQ u~(Q)
            out = np.stack([(E * (1j * Q[:, a] * ut)[None, :]) @ E.conj().T / self.nr for a in range(3)])
        self._mat[key] = out
        return out

    # ------------------------------------------------------------------ helpers
    def mom(self, *pairs):
        """Crystal momentum (fractional) of prod chi*_x phi_y over the given (x, y) pairs."""
        d = np.zeros(3)
        for x, y in pairs:
            d += self.kfrac[self.orbs[y]["k"]] - self.kfrac[self.orbs[x]["k"]]
        return d

    def gradu_conv(self, src, delta, ch):
        """[int dr' (grad u)(r - r') src(r')] for a scalar source -> (3,Nr)."""
        M = self.mat(delta, ch, "U")
        return np.stack([M[a] @ src for a in range(3)])

    def gradu_dot_conv(self, vsrc, delta, ch):
        """int dr' (grad u)(r - r') . vsrc(r') for a vector source (3,Nr) -> (Nr,)."""
        M = self.mat(delta, ch, "U")
        return sum(M[a] @ vsrc[a] for a in range(3))

    def periodic(self, j, full):
        """Cell-periodic part g_j of a full Bloch function of momentum k_j."""
        k = self.kfrac[self.orbs[j]["k"]] @ self.B
        return full * np.exp(-1j * self.r @ k) * math.sqrt(self.nk)

    # ------------------------------------------------------------------ two-body
    def two_body(self, j):
        """Literal h2 phi_j = sum_q f_q int dr2 chi*_q(r2) v2 [phi_j(r1)phi_q(r2) - phi_q(r1)phi_j(r2)]."""
        o = self.orbs
        sj = o[j]["s"]
        out = {t: 0 for t in ("2ah", "2bh1", "2bh2", "2ax", "2bx1", "2bx2")}
        for q in range(len(o)):
            sq, fq = o[q]["s"], o[q]["f"]
            ch = _pair(sj, sq)
            den = np.conj(o[q]["chi"]) * o[q]["phi"]
            out["2ah"] = out["2ah"] + fq * (self.mat(np.zeros(3), ch, "V", "H") @ den) * o[j]["phi"]
            h = self.gradu_conv(den, np.zeros(3), ch)
            # the Hartree-type vector kernel at Q = 0 is 0 in both conventions
            out["2bh1"] = out["2bh1"] + fq * np.sum(h * o[j]["grad"], 0)
            jsrc = np.conj(o[q]["chi"])[None] * o[q]["grad"]
            out["2bh2"] = out["2bh2"] - fq * self.gradu_dot_conv(jsrc, np.zeros(3), ch) * o[j]["phi"]
            if sq != sj:
                continue
            ex = np.conj(o[q]["chi"]) * o[j]["phi"]
            d = self.mom((q, j))
            out["2ax"] = out["2ax"] - fq * (self.mat(d, 0, "V", "X") @ ex) * o[q]["phi"]
            out["2bx1"] = out["2bx1"] - fq * np.sum(self.gradu_conv(ex, d, 0) * o[q]["grad"], 0)
            src = np.conj(o[q]["chi"])[None] * o[j]["grad"]
            out["2bx2"] = out["2bx2"] + fq * self.gradu_dot_conv(src, d, 0) * o[q]["phi"]
        return {t: self.periodic(j, v) for t, v in out.items()}

    # ------------------------------------------------------------------ three-body
    def three_body(self, j):
        """All 18 literal three-body integrals for target j: keys '3a1'..'3a6', '3b1'..'3b6', '3c1'..'3c6'."""
        o = self.orbs
        sj = o[j]["s"]
        out = {}
        for (nm, sign, perm), (q1, q2) in itertools.product(PERMS, itertools.product(range(len(o)), repeat=2)):
            labels = (j, q1, q2)
            a, b, c = (labels[perm[0]], labels[perm[1]], labels[perm[2]])
            spins = (sj, o[q1]["s"], o[q2]["s"])
            if o[a]["s"] != sj or o[b]["s"] != spins[1] or o[c]["s"] != spins[2]:
                continue
            wgt = sign * o[q1]["f"] * o[q2]["f"]
            s2 = np.conj(o[q1]["chi"]) * o[b]["phi"]          # bra/ket at x2
            s3 = np.conj(o[q2]["chi"]) * o[c]["phi"]          # bra/ket at x3
            d2 = self.mom((q1, b))
            d3 = self.mom((q2, c))
            # centre x1: grad_1 u_12 . grad_1 u_13
            I2 = self.gradu_conv(s2, d2, _pair(spins[0], spins[1]))
            I3 = self.gradu_conv(s3, d3, _pair(spins[0], spins[2]))
            va = np.sum(I2 * I3, 0) * o[a]["phi"]
            # centre x2: grad_2 u_21 . grad_2 u_23 ; (grad u)(r2 - r1) = -(grad u)(r1 - r2)
            I3b = self.gradu_conv(s3, d3, _pair(spins[1], spins[2]))
            vb = -self.gradu_dot_conv(s2[None] * I3b, d2 + d3, _pair(spins[1], spins[0])) * o[a]["phi"]
            # centre x3: grad_3 u_31 . grad_3 u_32
            I2c = self.gradu_conv(s2, d2, _pair(spins[2], spins[1]))
            vc = -self.gradu_dot_conv(s3[None] * I2c, d2 + d3, _pair(spins[2], spins[0])) * o[a]["phi"]
            for tag, v in (("3a", va), ("3b", vb), ("3c", vc)):
                out[tag + nm] = out.get(tag + nm, 0) + wgt * v
        return {t: self.periodic(j, v) for t, v in out.items()}
