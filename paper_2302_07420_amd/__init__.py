"""MI355X transcorrelated-operator library: thin Python binding of libtcmi.so.

Argument marshalling only: every step of the operator runs in the HIP library
(include/tcmi.h).  The library must have been built (``build.py``); importing
this package without it raises, there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libtcmi.so")

TC_PREC_FP64 = 0
TC_PREC_FP32 = 1
TC_PREC_FP32_SPLITBF16 = 2
# div_correction codes of tc_set_options (readings of the mesh divergence corrections)
TC_DIV_OFF = 0
TC_DIV_PRINTED = 1
TC_DIV_LIMIT = 2
_READINGS = {"printed": TC_DIV_PRINTED, "limit": TC_DIV_LIMIT}

TERM_BITS = {
    "2ah": 1 << 0, "2bh1": 1 << 1, "2bh2": 1 << 2, "2ax": 1 << 3, "2bx1": 1 << 4, "2bx2": 1 << 5,
    "3a1": 1 << 6, "3a2": 1 << 7, "3a3": 1 << 8, "3a4": 1 << 9, "3b1": 1 << 10, "3b2": 1 << 11,
    "3b3": 1 << 12, "3b4": 1 << 13, "3b5": 1 << 14, "3b6": 1 << 15, "corr": 1 << 16,
}
TERM_ALL = (1 << 17) - 1
E_PARTS = ("kinetic", "two_body", "three_body", "corrections")
# kernel index -> symbol stem (working precision R, grid length N), see TC_K_* in include/tcmi.h
KERNELS = ("k_scatter", "k_fft_xy<R,N,-1>", "k_fft_xy<R,N,1>", "k_fft_z<R,N,-1>", "k_fft_z<R,N,1>",
           "k_pair_xy<R,N,true>", "k_pair_xy<R,N,false>", "k_sum_parts<R,N>", "k_passB_xy<R,N>",
           "k_zconv<R,N,OP_O>", "k_zconv<R,N,OP_A1>", "k_zconv<R,N,OP_A2>", "k_zconv<R,N,OP_B>",
           "k_fused_O<R,N>", "k_fused_A<R,N>", "k_fused_Y<R,N>", "other", "fp64_corrections",
           "k_fused_OB<R,N>")
STAGES = ("g_to_r", "hartree", "occ_occ", "pass_a", "pass_b", "out_and_corrections")

_lib = None
# tc_set_allocator callbacks: void* alloc(size_t bytes, void* user); void free(void* p, size_t bytes, void* user)
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)


class TCError(RuntimeError):
    pass


class SCFParams(ctypes.Structure):
    """tc_scf_params of include/tcmi.h."""
    _fields_ = [("max_iter", ctypes.c_int), ("pmax", ctypes.c_int), ("etol", ctypes.c_double),
                ("mix", ctypes.c_double), ("otol", ctypes.c_double)]


def lib():
    """Load libtcmi.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        raise TCError(f"{LIBPATH} not found: build it with paper_2302_07420_amd/build.py")
    L = ctypes.CDLL(LIBPATH)
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    dp = ctypes.POINTER(ctypes.c_double)
    sig = {
        "tc_create": (I, [I, P, ctypes.POINTER(P)]),
        "tc_destroy": (None, [P]),
        "tc_last_error": (ctypes.c_char_p, [P]),
        "tc_set_cell": (I, [P, dp]),
        "tc_set_kmesh": (I, [P, I, I, I]),
        "tc_set_kmesh_shift": (I, [P, dp]),
        "tc_set_jastrow_cusp": (I, [P, dp]),
        "tc_set_grid": (I, [P, I, I, I]),
        "tc_set_basis": (I, [P, I, I, ctypes.POINTER(ctypes.c_int32)]),
        "tc_set_jastrow": (I, [P, dp, dp]),
        "tc_set_options": (I, [P, I, D, I, ctypes.c_uint64]),
        "tc_load_orbitals": (I, [P, I, I, dp, dp, dp]),
        "tc_set_nspin": (I, [P, I]),
        "tc_set_symmetry": (I, [P, I, ctypes.POINTER(ctypes.c_int32), dp]),
        "tc_set_band_kpoints": (I, [P, I, dp]),
        "tc_set_band_basis": (I, [P, I, I, ctypes.POINTER(ctypes.c_int32)]),
        "tc_load_band_orbitals": (I, [P, I, I, dp, dp]),
        "tc_apply_band": (I, [P, dp, dp]),
        "tc_load_orbitals_spin": (I, [P, I, I, I, dp, dp, dp]),
        "tc_orbital_energies": (I, [P, dp]),
        "tc_apply": (I, [P, I, dp, dp]),
        "tc_scf": (I, [P, ctypes.POINTER(SCFParams), dp, ctypes.POINTER(I)]),
        "tc_energy_backward_lr": (I, [P, dp, dp, dp, dp]),
        "tc_get_orbitals": (I, [P, I, dp, dp]),
        "tc_get_orbitals_spin": (I, [P, I, I, dp, dp]),
        "tc_apply_dev": (I, [P, I, P, P]),
        "tc_load_orbitals_dev": (I, [P, I, I, P, dp]),
        "tc_apply_all": (I, [P, dp]),
        "tc_apply_all_dev": (I, [P, P]),
        "tc_apply_all_dev_noalloc": (I, [P, P]),
        "tc_energy": (I, [P, dp, dp]),
        "tc_energy_backward": (I, [P, dp, dp, dp]),
        "tc_energy_backward_dev": (I, [P, P, dp, dp]),
        "tc_sync": (I, [P]),
        "tc_last_timing": (I, [P, dp, dp, I]),
        "tc_set_batch": (I, [P, I]),
        "tc_set_pair_store": (I, [P, I]),
        "tc_set_profiling": (I, [P, I]),
        "tc_kernel_stats": (I, [P, dp, dp, dp, I]),
        "tc_set_allocator": (I, [P, ALLOC_FN, FREE_FN, P]),
        "tc_set_memory_budget": (I, [P, ctypes.c_size_t]),
        "tc_get_stream": (P, [P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class TCOperator:
    """One problem on one device.  Mirrors the C ABI call for call."""

    def __init__(self, device: int = 0, stream: Optional[int] = None):
        self._L = lib()
        h = ctypes.c_void_p()
        st = self._L.tc_create(device, ctypes.c_void_p(stream) if stream else None, ctypes.byref(h))
        if st != 0:
            raise TCError(f"tc_create failed with status {st}")
        self._h = h
        self.npw: List[int] = []
        self.nband = 0
        self.nspin = 1

    def _check(self, st: int, what: str):
        if st != 0:
            msg = self._L.tc_last_error(self._h).decode()
            raise TCError(f"{what}: status {st}: {msg}")

    def close(self):
        if getattr(self, "_h", None):
            self._L.tc_destroy(self._h)
            self._h = None
        self._alloc_cb = None   # the allocator callbacks outlive the context

    def stream(self) -> int:
        """The hipStream_t (as an integer) the library enqueues this context's work on."""
        return int(self._L.tc_get_stream(self._h) or 0)

    def use_torch_allocator(self, device: int = 0):
        """Take every later device buffer of the context from PyTorch's caching allocator (on the context's
        stream), so that torch.cuda.memory_allocated() counts it; tc_destroy gives it back."""
        import torch

        stream = self.stream()

        def _alloc(nbytes, user):
            try:
                return torch.cuda.caching_allocator_alloc(int(nbytes), device, stream)
            except Exception:   # out of memory: the library reports TC_ERR_OOM
                return None

        def _free(ptr, nbytes, user):
            torch.cuda.caching_allocator_delete(ptr)

        cbs = (ALLOC_FN(_alloc), FREE_FN(_free))
        self._check(self._L.tc_set_allocator(self._h, cbs[0], cbs[1], None), "tc_set_allocator")
        self._alloc_cb = cbs

    def set_memory_budget(self, nbytes: int):
        self._check(self._L.tc_set_memory_budget(self._h, int(nbytes)), "tc_set_memory_budget")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------------- setters
    def set_cell(self, lattice):
        a = np.ascontiguousarray(np.asarray(lattice, dtype=np.float64).reshape(9))
        self._check(self._L.tc_set_cell(self._h, _dp(a)), "tc_set_cell")

    def set_kmesh(self, n1, n2, n3, shift=None):
        """n1 x n2 x n3 Monkhorst-Pack mesh; ``shift`` (3 components in [0, 1), mesh units) moves every
        k-point to (i + s) / n (tc_set_kmesh_shift)."""
        self._check(self._L.tc_set_kmesh(self._h, n1, n2, n3), "tc_set_kmesh")
        self.npw = [0] * (n1 * n2 * n3)
        if shift is not None and any(float(x) != 0.0 for x in shift):
            self.set_kmesh_shift(shift)

    def set_kmesh_shift(self, shift):
        s = np.ascontiguousarray(np.asarray(shift, dtype=np.float64).reshape(3))
        self._check(self._L.tc_set_kmesh_shift(self._h, _dp(s)), "tc_set_kmesh_shift")

    def set_jastrow_cusp(self, A):
        """A (parallel, antiparallel) with C from the cusp conditions (tc_set_jastrow_cusp)."""
        a = np.ascontiguousarray(np.asarray(A, dtype=np.float64).reshape(2))
        self._check(self._L.tc_set_jastrow_cusp(self._h, _dp(a)), "tc_set_jastrow_cusp")

    def set_grid(self, N1, N2, N3):
        self._check(self._L.tc_set_grid(self._h, N1, N2, N3), "tc_set_grid")

    def set_basis(self, ik, miller):
        m = np.ascontiguousarray(np.asarray(miller, dtype=np.int32).reshape(-1, 3))
        self._check(self._L.tc_set_basis(self._h, ik, m.shape[0], m.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))),
                    "tc_set_basis")
        self.npw[ik] = m.shape[0]

    def set_jastrow(self, A, C):
        a = np.ascontiguousarray(np.asarray(A, dtype=np.float64))
        c = np.ascontiguousarray(np.asarray(C, dtype=np.float64))
        self._check(self._L.tc_set_jastrow(self._h, _dp(a), _dp(c)), "tc_set_jastrow")

    def set_options(self, precision=TC_PREC_FP64, alpha=1.0, div_correction=True, terms=TERM_ALL,
                    reading="printed"):
        """div_correction on/off; reading "printed" (TC_DIV_PRINTED) or "limit" (TC_DIV_LIMIT)."""
        if reading not in _READINGS:
            raise ValueError("reading must be 'printed' or 'limit'")
        code = _READINGS[reading] if div_correction else TC_DIV_OFF
        self._check(self._L.tc_set_options(self._h, int(precision), float(alpha), code, int(terms)),
                    "tc_set_options")

    def set_nspin(self, nspin: int):
        """1: both spin channels hold the same orbitals; 2: spin-polarised TC mode (load spin 1 separately)."""
        self._check(self._L.tc_set_nspin(self._h, int(nspin)), "tc_set_nspin")
        self.nspin = int(nspin)

    def set_symmetry(self, ops=None):
        """Crystal symmetry: ``ops`` a list of (R (3,3) int, tau (3,)) with x -> R (x + tau) on fractional
        coordinates; None or [] switches it off.  Only the representative k-points' orbitals are used."""
        if not ops:
            self._check(self._L.tc_set_symmetry(self._h, 0, None, None), "tc_set_symmetry")
            return
        rot = np.ascontiguousarray(np.stack([np.asarray(R, dtype=np.int32) for R, _ in ops]))
        tau = np.ascontiguousarray(np.stack([np.asarray(t, dtype=np.float64) for _, t in ops]))
        self._check(self._L.tc_set_symmetry(self._h, len(ops), rot.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                            _dp(tau)), "tc_set_symmetry")

    def set_band(self, kpoints, millers, coeffs, occs):
        """Band (zero-weight) k-points: fractional k (nkb, 3), per band k-point its Miller set, orbitals
        (nband, npw) and fillings."""
        k = np.ascontiguousarray(np.asarray(kpoints, dtype=np.float64).reshape(-1, 3))
        self._check(self._L.tc_set_band_kpoints(self._h, k.shape[0], _dp(k)), "tc_set_band_kpoints")
        self.band_npw = []
        for ib, m in enumerate(millers):
            mm = np.ascontiguousarray(np.asarray(m, dtype=np.int32).reshape(-1, 3))
            self._check(self._L.tc_set_band_basis(self._h, ib, mm.shape[0],
                                                  mm.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))), "tc_set_band_basis")
            self.band_npw.append(mm.shape[0])
        for ib, (c, o) in enumerate(zip(coeffs, occs)):
            cc = np.ascontiguousarray(np.asarray(c, dtype=np.complex128))
            oo = np.ascontiguousarray(np.asarray(o, dtype=np.float64))
            self._check(self._L.tc_load_band_orbitals(self._h, ib, cc.shape[0], _dp(cc.view(np.float64)), _dp(oo)),
                        "tc_load_band_orbitals")
            self.band_nb = cc.shape[0]

    def apply_band(self):
        """(H c per band k-point as (nband, npw) arrays, orbital energies [nkb, nband])."""
        nkb, nb, npm = len(self.band_npw), self.band_nb, max(self.band_npw)
        out = np.zeros((nkb, nb, npm), dtype=np.complex128)
        eps = np.zeros((nkb, nb), dtype=np.complex128)
        self._check(self._L.tc_apply_band(self._h, _dp(out.view(np.float64)), _dp(eps.view(np.float64))),
                    "tc_apply_band")
        return [out[b, :, : self.band_npw[b]].copy() for b in range(nkb)], eps

    def load_orbitals(self, ik, coeff, occ, left=None, spin=0):
        """Right orbitals ``coeff`` (nband, npw) of k-point ik; ``left`` (same shape) switches that k-point to
        the biorthogonal mode (the library normalises the right set and biorthogonalises the left one).
        ``spin`` = 1 loads the spin-down channel of a spin-polarised problem (after set_nspin(2))."""
        c = np.ascontiguousarray(np.asarray(coeff, dtype=np.complex128))
        o = np.ascontiguousarray(np.asarray(occ, dtype=np.float64))
        lp = None
        if left is not None:
            lc = np.ascontiguousarray(np.asarray(left, dtype=np.complex128))
            if lc.shape != c.shape:
                raise ValueError("left and right coefficient arrays differ in shape")
            lp = _dp(lc.view(np.float64))
        self.nband = c.shape[0]
        if spin:
            self._check(self._L.tc_load_orbitals_spin(self._h, int(spin), ik, c.shape[0], _dp(c.view(np.float64)),
                                                      lp, _dp(o)), "tc_load_orbitals_spin")
            return
        self._check(self._L.tc_load_orbitals(self._h, ik, c.shape[0], _dp(c.view(np.float64)), lp, _dp(o)),
                    "tc_load_orbitals")

    def load_orbitals_dev(self, ik, ptr: int, nband: int, occ):
        o = np.ascontiguousarray(np.asarray(occ, dtype=np.float64))
        self.nband = nband
        self._check(self._L.tc_load_orbitals_dev(self._h, ik, nband, ctypes.c_void_p(ptr), _dp(o)),
                    "tc_load_orbitals_dev")

    # ---------------------------------------------------------------- work
    @property
    def npw_max(self):
        return max(self.npw) if self.npw else 0

    def apply(self):
        """(H c) per k-point as (nband, npw) arrays; with two spin channels, one such list per spin."""
        nk = len(self.npw)
        if nk == 0 or self.npw_max == 0 or self.nband == 0:
            # let the library report the missing set-up (TC_ERR_STATE)
            self._check(self._L.tc_apply_all(self._h, None), "tc_apply_all")
        out = np.zeros((self.nspin, nk, self.nband, self.npw_max), dtype=np.complex128)
        self._check(self._L.tc_apply_all(self._h, _dp(out.view(np.float64))), "tc_apply_all")
        per = [[out[s, k, :, : self.npw[k]] for k in range(nk)] for s in range(self.nspin)]
        return per[0] if self.nspin == 1 else per

    def apply_dev(self, out_ptr: Optional[int] = None):
        self._check(self._L.tc_apply_all_dev(self._h, ctypes.c_void_p(out_ptr) if out_ptr else None),
                    "tc_apply_all_dev")

    def apply_dev_noalloc(self, out_ptr: int):
        """tc_apply_all_dev_noalloc: the same application with every device buffer from the library's fixed
        scratch (needs one ordinary application on this context since its last change)."""
        self._check(self._L.tc_apply_all_dev_noalloc(self._h, ctypes.c_void_p(out_ptr)), "tc_apply_all_dev_noalloc")

    def energy(self):
        e = np.zeros(1)
        parts = np.zeros(len(E_PARTS))
        self._check(self._L.tc_energy(self._h, _dp(e), _dp(parts)), "tc_energy")
        return float(e[0]), dict(zip(E_PARTS, parts.tolist()))

    def apply_vectors(self, vecs) -> List[np.ndarray]:
        """h v for trial vectors: ``vecs`` per k-point (nvec, npw(k)), the same nvec everywhere; with two spin
        channels, one such list per channel (each against its own channel's operator)."""
        nk, ns = len(self.npw), self.nspin
        per = [vecs] if ns == 1 else list(vecs)
        nvec = np.asarray(per[0][0]).shape[0]
        buf = np.zeros((ns, nk, nvec, self.npw_max), dtype=np.complex128)
        for sp in range(ns):
            for k in range(nk):
                v = np.asarray(per[sp][k], dtype=np.complex128)
                if v.shape != (nvec, self.npw[k]):
                    raise ValueError(f"k-point {k}: vectors of shape {v.shape}, expected {(nvec, self.npw[k])}")
                buf[sp, k, :, : self.npw[k]] = v
        out = np.zeros_like(buf)
        self._check(self._L.tc_apply(self._h, nvec, _dp(buf.view(np.float64)), _dp(out.view(np.float64))),
                    "tc_apply")
        res = [[out[sp, k, :, : self.npw[k]].copy() for k in range(nk)] for sp in range(ns)]
        return res[0] if ns == 1 else res

    def apply_vectors_dev(self, nvec: int, in_ptr: int, out_ptr: int):
        """Device form of apply_vectors: [nk][nvec][npw_max] complex128 buffers (synchronous)."""
        self._check(self._L.tc_apply_dev(self._h, int(nvec), ctypes.c_void_p(in_ptr), ctypes.c_void_p(out_ptr)),
                    "tc_apply_dev")

    def scf(self, max_iter=50, pmax=2, etol=1e-10, mix=1.0, otol=1e-8):
        """Block-Davidson TC / BITC self-consistent loop; returns (energies per iteration, iterations)."""
        prm = SCFParams(int(max_iter), int(pmax), float(etol), float(mix), float(otol))
        e = np.zeros(max(1, int(max_iter)))
        n = ctypes.c_int(0)
        self._check(self._L.tc_scf(self._h, ctypes.byref(prm), _dp(e), ctypes.byref(n)), "tc_scf")
        return e[: n.value].copy(), n.value

    def get_orbitals(self, ik, left=False, spin=None):
        """Current orbitals of k-point ik: right (nband, npw), and left too when ``left``; ``spin`` selects the
        channel with two spin channels."""
        r = np.zeros((self.nband, self.npw[ik]), dtype=np.complex128)
        l = np.zeros_like(r) if left else None
        if spin is None:
            self._check(self._L.tc_get_orbitals(self._h, int(ik), _dp(r.view(np.float64)),
                                                _dp(l.view(np.float64)) if left else None), "tc_get_orbitals")
        else:
            self._check(self._L.tc_get_orbitals_spin(self._h, int(spin), int(ik), _dp(r.view(np.float64)),
                                                     _dp(l.view(np.float64)) if left else None),
                        "tc_get_orbitals_spin")
        return (r, l) if left else r

    def orbital_energies(self) -> np.ndarray:
        """Complex eps_j = <chi_j| T + h |phi_j> per orbital of the last application, shape [nk, nband]
        ([2, nk, nband] with two spin channels)."""
        e = np.zeros(self.nspin * len(self.npw) * self.nband, dtype=np.complex128)
        self._check(self._L.tc_orbital_energies(self._h, _dp(e.view(np.float64))), "tc_orbital_energies")
        shape = (len(self.npw), self.nband) if self.nspin == 1 else (2, len(self.npw), self.nband)
        return e.reshape(shape)

    def backward(self, want_grad=True, want_params=True):
        """(grad per k as (nband, npw) complex128 = 2 dE/dc*, dE/dA (2,), dE/dC (2,)); unrequested parts are None.
        With two spin channels grad is [per k of spin 0, per k of spin 1]."""
        nk, ns = len(self.npw), self.nspin
        g = np.zeros((ns * nk, self.nband, self.npw_max), dtype=np.complex128) if want_grad else None
        dA = np.zeros(2) if want_params else None
        dC = np.zeros(2) if want_params else None
        self._check(self._L.tc_energy_backward(self._h, _dp(g.view(np.float64)) if want_grad else None,
                                               _dp(dA) if want_params else None, _dp(dC) if want_params else None),
                    "tc_energy_backward")
        if not want_grad:
            return None, dA, dC
        per = [[g[sp * nk + k, :, : self.npw[k]] for k in range(nk)] for sp in range(ns)]
        return (per[0] if ns == 1 else per), dA, dC

    def backward_lr(self, want_right=True, want_left=True, want_params=True):
        """(grad_right, grad_left, dA, dC); biorthogonal mode: the two partial gradients (TC mode: the
        gradient as grad_right and want_left must be False).  With two spin channels each gradient is
        [per k of spin 0, per k of spin 1]."""
        nk, ns = len(self.npw), self.nspin
        gr = np.zeros((ns * nk, self.nband, self.npw_max), dtype=np.complex128) if want_right else None
        gl = np.zeros((ns * nk, self.nband, self.npw_max), dtype=np.complex128) if want_left else None
        dA = np.zeros(2) if want_params else None
        dC = np.zeros(2) if want_params else None
        self._check(self._L.tc_energy_backward_lr(self._h, None if gr is None else _dp(gr.view(np.float64)),
                                                  None if gl is None else _dp(gl.view(np.float64)),
                                                  None if dA is None else _dp(dA), None if dC is None else _dp(dC)),
                    "tc_energy_backward_lr")
        def cut(g):
            if g is None:
                return None
            per = [[g[sp * nk + k, :, : self.npw[k]].copy() for k in range(nk)] for sp in range(ns)]
            return per[0] if ns == 1 else per

        return cut(gr), cut(gl), dA, dC

    def backward_dev(self, grad_ptr: Optional[int], want_params=True):
        """Gradient into a device buffer [nk][nband][npw_max] complex128; returns (dE/dA, dE/dC) or (None, None)."""
        dA = np.zeros(2) if want_params else None
        dC = np.zeros(2) if want_params else None
        self._check(self._L.tc_energy_backward_dev(self._h, ctypes.c_void_p(grad_ptr) if grad_ptr else None,
                                                   _dp(dA) if want_params else None,
                                                   _dp(dC) if want_params else None), "tc_energy_backward_dev")
        return dA, dC

    def sync(self):
        self._check(self._L.tc_sync(self._h), "tc_sync")

    def set_batch(self, targets_per_batch: int):
        self._check(self._L.tc_set_batch(self._h, int(targets_per_batch)), "tc_set_batch")

    def set_pair_store(self, on: bool):
        self._check(self._L.tc_set_pair_store(self._h, int(bool(on))), "tc_set_pair_store")

    def set_profiling(self, on: bool):
        self._check(self._L.tc_set_profiling(self._h, int(bool(on))), "tc_set_profiling")

    def kernel_stats(self, reset: bool = False):
        n = len(KERNELS)
        ms, cnt, by = np.zeros(n), np.zeros(n), np.zeros(n)
        self._check(self._L.tc_kernel_stats(self._h, _dp(ms), _dp(cnt), _dp(by), int(reset)), "tc_kernel_stats")
        return {f: dict(ms=float(ms[i]), launches=int(cnt[i]), bytes=float(by[i])) for i, f in enumerate(KERNELS)}

    def timing(self):
        tot = np.zeros(1)
        st = np.zeros(6)
        self._check(self._L.tc_last_timing(self._h, _dp(tot), _dp(st), 6), "tc_last_timing")
        return float(tot[0]), st.tolist()


def from_workload(w, precision=TC_PREC_FP64, terms=TERM_ALL, div_correction=True, device=0, A=None, C=None,
                  coeff=None, stream=None, batch=0, left=None, symmetry=None, pair_store=True,
                  reading="printed", torch_alloc=False, mem_budget=0) -> TCOperator:
    """Build an operator from a ``tcinputs.Workload``: TC mode, or the biorthogonal mode when the workload
    (or ``left``) holds left orbitals; ``symmetry``: crystal operations [(R, tau)] (see set_symmetry);
    ``torch_alloc``: device memory from PyTorch's caching allocator; ``mem_budget``: bytes for the pair
    store and pair buffers (tc_set_memory_budget)."""
    op = TCOperator(device, stream)
    if torch_alloc:
        op.use_torch_allocator(device)
    if mem_budget:
        op.set_memory_budget(mem_budget)
    if batch:
        op.set_batch(batch)
    if not pair_store:
        op.set_pair_store(False)
    op.set_cell(w.lattice)
    op.set_kmesh(*w.kmesh, shift=getattr(w, "kshift", None))
    op.set_grid(*w.grid)
    for ik, m in enumerate(w.miller):
        op.set_basis(ik, m)
    op.set_jastrow(w.A if A is None else A, w.C if C is None else C)
    op.set_options(precision, w.alpha, div_correction, terms, reading)
    if symmetry:
        op.set_symmetry(symmetry)
    cs = w.right if coeff is None else coeff
    ls = w.left if left is None else left
    dn = getattr(w, "right_dn", None)
    ldn = getattr(w, "left_dn", None)
    if dn is not None:   # spin-polarised workload (left orbitals of the down channel: biorthogonal mode)
        op.set_nspin(2)
    for ik in range(len(w.miller)):
        op.load_orbitals(ik, cs[ik], w.occ[ik], None if ls is None else ls[ik])
        if dn is not None:
            occd = w.occ_dn if w.occ_dn is not None else w.occ
            op.load_orbitals(ik, dn[ik], occd[ik], None if ldn is None else ldn[ik], spin=1)
    if getattr(w, "band_k", None) is not None:
        op.set_band(w.band_k, w.band_miller, w.band_right, w.band_occ)
    return op


def energy_function():
    """torch.autograd.Function for E(c, A, C) of an operator's problem (TC mode).

    ``TCEnergy.apply(op, coeff, A, C, occ)``: ``coeff`` is a complex128 CUDA tensor
    [nk, nband, npw_max] (rows zero-padded like tc_apply_all), ``A`` and ``C`` float64
    tensors of shape (2,), ``occ`` a float64 array [nk, nband].  Forward loads the
    coefficients and Jastrow parameters into ``op`` and returns the energy (float64
    scalar); backward loads the same inputs again (the op may hold others by then) and
    calls tc_energy_backward_dev, whose gradient convention
    (dE/dRe c + i dE/dIm c) is the one torch uses for complex leaves.  Only argument
    marshalling happens here; the energy and its gradient are computed by the library.
    """
    import torch

    def load(op, coeff, A, C, occ):
        nk, nb, npw_max = coeff.shape
        op.set_jastrow(A.detach().cpu().numpy(), C.detach().cpu().numpy())
        packed = [coeff[k, :, : op.npw[k]].contiguous() for k in range(nk)]   # [nband][npw(k)] rows
        torch.cuda.current_stream().synchronize()
        for k in range(nk):
            op.load_orbitals_dev(k, packed[k].data_ptr(), nb, occ[k])
        op.sync()

    class TCEnergy(torch.autograd.Function):
        @staticmethod
        def forward(ctx, op, coeff, A, C, occ):
            if coeff.dtype != torch.complex128 or not coeff.is_cuda or not coeff.is_contiguous():
                raise TCError("coeff must be a contiguous complex128 CUDA tensor [nk, nband, npw_max]")
            nk, nb, npw_max = coeff.shape
            if npw_max != op.npw_max or nk != len(op.npw):
                raise TCError("coeff shape does not match the operator's k-mesh and basis")
            occ = np.asarray(occ, dtype=np.float64).reshape(nk, nb)
            load(op, coeff, A, C, occ)
            e, _ = op.energy()
            ctx.op = op
            ctx.occ = occ
            ctx.save_for_backward(coeff.detach(), A.detach(), C.detach())
            return torch.tensor(e, dtype=torch.float64)

        @staticmethod
        def backward(ctx, gE):
            # the op may have been loaded with other inputs since this forward (a second forward, gradcheck):
            # load this forward's coefficients and Jastrow parameters again before the gradient
            coeff, A, C = ctx.saved_tensors
            load(ctx.op, coeff, A, C, ctx.occ)
            grad = torch.zeros(coeff.shape, dtype=torch.complex128, device=coeff.device)
            torch.cuda.current_stream().synchronize()
            dA, dC = ctx.op.backward_dev(grad.data_ptr())
            g = float(gE)
            return (None, grad * g, torch.as_tensor(dA * g, dtype=torch.float64, device=A.device),
                    torch.as_tensor(dC * g, dtype=torch.float64, device=C.device), None)

    return TCEnergy
