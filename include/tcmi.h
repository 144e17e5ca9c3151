/* tcmi.h - C ABI of the MI355X transcorrelated-operator library.
 *
 * The library applies the two- and three-body terms of the transcorrelated
 * (TC) effective one-body operator h of arXiv:2302.07420 (Sec. 2.1, Eq. SCF;
 * terms of Secs. 2.6.3-2.6.4) to every occupied orbital of a spin-unpolarized
 * plane-wave problem on a uniform Gamma-centred k-mesh, by the FFT pair-density
 * route of the paper's algorithms (Algs. 2ah, 2ax, 3a1-3a4, 3b1-3b6) with the
 * Gygi-Baldereschi divergence corrections for k-points on the SCF mesh
 * (Sec. 2.5; Eqs. divcorr_2ax_scf, divcor_3a2_first/second in their
 * general-overlap form, 3b6_div_scf1-3).  It also returns the TC pseudo-energy
 * (Eq. EtotTC) and its gradient with respect to the orbital coefficients and
 * the Jastrow parameters A and C of Eq. Jastrow.  With left orbitals loaded it
 * works in the biorthogonal mode (BITC, Sec. 2.3, Eqs. BITCSCF and EtotBiTC):
 * every bra, density and overlap takes conj(chi) in place of conj(phi).
 *
 * Conventions shared by every call
 *  - All calls return an int status: TC_OK (0) or a negative TC_ERR_* code;
 *    tc_last_error() then describes the failure.  No exception crosses the ABI.
 *  - A context is not internally synchronised: use one context per thread.
 *  - Lattice rows a1, a2, a3 are in bohr; reciprocal rows b_j satisfy
 *    a_i . b_j = 2 pi delta_ij.  k-point ik = (i1*n2 + i2)*n3 + i3 sits at
 *    k = (i1/n1, i2/n2, i3/n3) in units of b (Gamma-centred mesh).
 *  - Orbital coefficients c(G) are complex128, interleaved (re, im), band-major:
 *    [band][npw(ik)], for the cell-periodic part phi(r) = Omega^{-1/2}
 *    sum_G c(G) e^{iG.r} (Sec. 2.3 with sum |c|^2 = 1).  G = m1 b1 + m2 b2 + m3 b3
 *    with the Miller indices given to tc_set_basis.
 *  - Host buffers passed in are only read during the call (borrowed); host
 *    output buffers are written before the call returns.  Device pointers
 *    (the *_dev calls) belong to the caller, are read/written in stream order on
 *    the context's stream and must stay alive until that stream reaches the
 *    work; call tc_sync() to wait.
 *  - Energies are in hartree per cell, summed over both spin channels.
 */
#ifndef TCMI_H
#define TCMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tc_ctx tc_ctx;

enum {
  TC_OK = 0,
  TC_ERR_ARG = -1,          /* invalid argument (null pointer, out-of-range value)  */
  TC_ERR_STATE = -2,        /* call made before a required setter                    */
  TC_ERR_GRID = -3,         /* a plane wave does not fit the FFT grid                */
  TC_ERR_KMESH = -4,        /* k-mesh / basis inconsistent                           */
  TC_ERR_UNSUPPORTED = -5,  /* grid size, mode or option not implemented             */
  TC_ERR_DEVICE = -6,       /* HIP runtime error                                      */
  TC_ERR_OOM = -7           /* device allocation failed                              */
};

enum {
  TC_PREC_FP64 = 0,             /* everything in FP64                                                */
  TC_PREC_FP32 = 1,             /* FP32 FFT butterflies, pair products and kernel multiplies          */
  TC_PREC_FP32_SPLITBF16 = 2    /* as FP32, with the DFTs along z as dense GEMMs on the matrix cores in
                                   split BF16 (hi + lo, three products, FP32 accumulation); grid
                                   lengths divisible by 8, else TC_ERR_UNSUPPORTED at application   */
};

/* Term selection bits for tc_set_options (names follow Sec. 2.6 of the paper).
 * Three-body terms enter the operator with multiplicity 2 for 3a3, 3a4 and all
 * 3b terms (3a6 = 3a3, 3a5 = 3a4, 3c* = 3b*).  TC_T_CORR enables the SCF-mesh
 * divergence corrections of the selected terms (2ax, 3a2, 3b6). */
enum {
  TC_T_2AH = 1 << 0, TC_T_2BH1 = 1 << 1, TC_T_2BH2 = 1 << 2,
  TC_T_2AX = 1 << 3, TC_T_2BX1 = 1 << 4, TC_T_2BX2 = 1 << 5,
  TC_T_3A1 = 1 << 6, TC_T_3A2 = 1 << 7, TC_T_3A3 = 1 << 8, TC_T_3A4 = 1 << 9,
  TC_T_3B1 = 1 << 10, TC_T_3B2 = 1 << 11, TC_T_3B3 = 1 << 12, TC_T_3B4 = 1 << 13,
  TC_T_3B5 = 1 << 14, TC_T_3B6 = 1 << 15,
  TC_T_CORR = 1 << 16,
  TC_T_ALL = (1 << 17) - 1
};

/* div_correction values of tc_set_options.
 * TC_DIV_PRINTED: the SCF-mesh corrections as printed: the G = G' = 0 corrections of 3a2 and 3b6
 *   (Eqs. divcor_3a2_first, 3b6_div_scf1) carry one u~_short(0)/N_k (Eq. u_short), and 2bx1 has none.
 * TC_DIV_LIMIT: the mesh operator taken as the limit of the band operator at a mesh point: two
 *   u~_short(0)/N_k in those corrections (the whole finite Q -> 0 remainder of Q^2 u~(Q)^2), and on
 *   2bx1 the remainder -(4 pi A_par / N_k) sum_mu f_mu FT[chi*_mu phi_j](0) phi_mu that the gradient
 *   leaves on the partner's Bloch phase (mu over the target's k-point).
 * The band forms (band k-points) are the same in both. */
enum { TC_DIV_OFF = 0, TC_DIV_PRINTED = 1, TC_DIV_LIMIT = 2 };

/* Energy breakdown written by tc_energy (hartree per cell, both spins). */
enum {
  TC_E_KINETIC = 0,   /* sum f <chi|-lap/2|phi> / N_k (chi = phi in TC mode)             */
  TC_E_TWO_BODY = 1,  /* (1/2) <h2>, h2 = 2ah+2bh1+2bh2+2ax+2bx1+2bx2 (+2ax correction)   */
  TC_E_THREE_BODY = 2,/* (1/3) <h3>, three-body terms with multiplicities (+ corrections)  */
  TC_E_CORR = 3,      /* part of the two entries above that comes from the corrections    */
  TC_E_NPARTS = 4
};

/* Create a context on HIP device `device`.  `stream` is a hipStream_t owned by
 * the caller (NULL: the library creates and owns one).  Allocates nothing large
 * until orbitals are loaded.  TC_ERR_DEVICE if the device is unusable. */
int tc_create(int device, void* stream, tc_ctx** out);

/* Device memory of the context from the caller (the memory the problem statement leaves to PyTorch):
 * every device buffer the library makes after this call comes from alloc_fn(bytes, user) and goes back
 * through free_fn(p, bytes, user) (bytes as allocated).  The context's stream is drained before a
 * buffer is given back.  Buffers made earlier keep the allocator that made them (hipMalloc before any
 * call).  alloc_fn returning NULL is TC_ERR_OOM at the call that needed the memory.  Both NULL: hipMalloc
 * again; one NULL: TC_ERR_ARG.  The functions and `user` must stay valid until tc_destroy. */
int tc_set_allocator(tc_ctx* ctx, void* (*alloc_fn)(size_t bytes, void* user),
                     void (*free_fn)(void* p, size_t bytes, void* user), void* user);

/* Bytes of device memory the resident pair store and the per-batch pair buffers (the two large
 * consumers) may take together; 0 (the default) sizes them from the device's memory.  With a budget the
 * store takes the partner columns that fit beside a batch of 8 targets (tc_set_pair_store), and the
 * batches take what it leaves (at most 32 GiB).  The next application resizes.  Results do not depend
 * on it. */
int tc_set_memory_budget(tc_ctx* ctx, size_t bytes);

/* The hipStream_t the context enqueues its work on (the caller's, or the one it created). */
void* tc_get_stream(const tc_ctx* ctx);

/* Release every device buffer and the owned stream.  NULL is ignored. */
void tc_destroy(tc_ctx* ctx);

/* Text of the last error on this context (owned by ctx, valid until the next call). */
const char* tc_last_error(const tc_ctx* ctx);

/* Lattice rows a1, a2, a3 (bohr); Omega = |det| must be > 0 (TC_ERR_ARG). */
int tc_set_cell(tc_ctx* ctx, const double lattice[9]);

/* Uniform Gamma-centred Monkhorst-Pack mesh n1 x n2 x n3 (Sec. 2.5 assumes a
 * uniform SCF mesh).  Each n_i in [1, 16]. */
int tc_set_kmesh(tc_ctx* ctx, int n1, int n2, int n3);

/* FFT grid.  The library supports cubic grids N1 = N2 = N3 = N with
 * N in {8, 12, 16, 24, 32, 48}; anything else is TC_ERR_UNSUPPORTED. */
/* Monkhorst-Pack shift of the k-mesh (Sec. "Functionalities" of the TC++ description: meshes with or
 * without a shift): k-point (i1, i2, i3) becomes ((i + s) / n) in units of the reciprocal rows, shift s in
 * mesh units, each component in [0, 1) (0: Gamma-centred, the default; 1/2: the shift of an even mesh).
 * Pair shifts k - q and the Gygi-Baldereschi constant do not change; the kinetic energy, the gradient
 * fields and band corrections use the shifted points.  Call after tc_set_kmesh (which resets it to 0) and
 * before the plane-wave sets (built by the caller for the shifted points); it discards loaded orbitals and
 * symmetry.  TC_ERR_STATE before the k-mesh, TC_ERR_ARG for a null or out-of-range shift.  Symmetry
 * operations must map the shifted mesh onto itself (TC_ERR_ARG from tc_set_symmetry otherwise). */
int tc_set_kmesh_shift(tc_ctx* ctx, const double shift[3]);

int tc_set_grid(tc_ctx* ctx, int N1, int N2, int N3);

/* Plane-wave set of k-point ik: npw Miller triples (m1,m2,m3) (int32, [npw][3]).
 * TC_ERR_GRID if a triple does not fit the grid (|m_i| >= N/2); TC_ERR_ARG if a triple
 * appears twice.  The grid should also satisfy N/2 >= 2 max|m_i| + 1 for alias-free pair
 * densities (not checked).  This and the other calls that only describe the problem
 * (cell, k-mesh, grid, Jastrow, options, spin channels, symmetry, band k-points, batch,
 * memory budget, profiling) do no device work. */
int tc_set_basis(tc_ctx* ctx, int ik, int npw, const int32_t* miller);

/* Jastrow parameters of Eq. Jastrow: index 0 = parallel spins, 1 = antiparallel.
 * A >= 0 (A = 0 gives Hartree-Fock), C > 0.  The cusp relation of Eq. cusp is
 * the caller's choice (A and C are independent here). */
int tc_set_jastrow(tc_ctx* ctx, const double A[2], const double C[2]);

/* tc_set_jastrow with C from the cusp conditions of Eq. cusp: C_par = sqrt(2 A_par), C_anti = sqrt(A_anti).
 * A > 0 (TC_ERR_ARG otherwise).  The gradients (tc_energy_backward*) stay the partial derivatives with the
 * four parameters independent; along the cusp-tied line dE/dA_s + dE/dC_s dC_s/dA_s is the total one. */
int tc_set_jastrow_cusp(tc_ctx* ctx, const double A[2]);

/* precision: TC_PREC_FP64, TC_PREC_FP32 or TC_PREC_FP32_SPLITBF16 (FFT butterflies,
 * pair products and kernel multiplies in that precision; corrections, overlaps,
 * partner sums across chunks and energy reductions always FP64).
 * alpha: exponent of the auxiliary function exp(-alpha q^2)/q^2 of Eq. aux (bohr^2, > 0).
 * div_correction: one of TC_DIV_* (the divergence corrections of Sec. 2.5 and their reading).
 * term_mask: OR of TC_T_* bits.  TC_ERR_ARG for any other precision or div_correction value. */
int tc_set_options(tc_ctx* ctx, int precision, double alpha, int div_correction, uint64_t term_mask);

/* Copy the occupied orbitals of k-point ik to the device: `right` holds nband x
 * npw(ik) complex128 coefficients, `occ` nband fillings per spin-orbital in [0, 1].
 * nband must be the same for every k-point.
 * left == NULL: TC mode (chi = phi); the coefficients are used as given.
 * left != NULL (same layout as right): biorthogonal mode for this k-point.  The
 *   library makes the pair biorthonormal in FP64 on the device, as Sec. 2.3
 *   requires (<chi_i|phi_j> = delta_ij, <phi_i|phi_i> = 1): each right orbital is
 *   normalised, S_ij = <chi_i|phi_j> is formed and inverted (Gauss-Jordan with
 *   partial pivoting) and the left set becomes conj(S^-1) chi.  TC_ERR_ARG if a
 *   right orbital is zero or S is singular (a pivot not above 1e-13 max|S_ij|); the
 *   k-point is then left unloaded.  Either every k-point or none must have left
 *   orbitals when the operator is applied (else TC_ERR_STATE).  The gradients of
 *   the biorthogonal mode are those of tc_energy_backward_lr. */
int tc_load_orbitals(tc_ctx* ctx, int ik, int nband, const double* right, const double* left,
                     const double* occ);

/* Same, TC mode, from a device buffer (complex128, [nband][npw(ik)]); occ stays on the host. */
int tc_load_orbitals_dev(tc_ctx* ctx, int ik, int nband, const void* right_dev, const double* occ);

/* Number of spin channels (Sec. 2.1 and Eq. SCF: one orbital set per spin; Sec. 2.6 sums every
 * Hartree-type field over both spins with the Jastrow channel u^{s s'} of the pair).  nspin = 1
 * (default): both channels hold the orbitals of tc_load_orbitals.  nspin = 2: spin-polarised, in TC mode or
 * (left orbitals in both channels) the biorthogonal mode; the spin-down set is loaded with
 * tc_load_orbitals_spin(ctx, 1, ...), the spin-up set with
 * tc_load_orbitals or spin 0.  Both channels have the same nband; exchange-type terms pair orbitals of
 * one spin, the parallel channel serves the own spin's density and partners and the antiparallel channel
 * the other spin's.  Outputs become spin-major: tc_apply_all* writes [2][nk][nband][npw_max] and
 * tc_orbital_energies [2][nk][nband] complex128; tc_energy sums both channels.  Call after the k-mesh;
 * it discards every loaded orbital.  Every call of the application, the energy, the trial vectors
 * (tc_apply*), the SCF loop and the gradients takes both channels; symmetry and band k-points are built
 * for one channel.
 * TC_ERR_ARG unless nspin is 1 or 2; TC_ERR_STATE before the k-mesh. */
int tc_set_nspin(tc_ctx* ctx, int nspin);

/* Band (zero-weight) k-points (Sec. 2.5 and the band forms of Sec. 2.6): k-points anywhere, not on the
 * SCF mesh, whose orbitals are targets of the operator of the loaded (mesh) orbitals and partners of none.
 * kfrac: nkb fractional k-points (units of the reciprocal rows, no reduction); 0 <= nkb <= 4096.  Call
 * after the k-mesh; it discards the band bases and orbitals; setting the k-mesh again removes them.
 * TC_ERR_ARG for a bad count or null k-points, TC_ERR_STATE before the k-mesh. */
int tc_set_band_kpoints(tc_ctx* ctx, int nkb, const double* kfrac);

/* Plane-wave set of band k-point ib (as tc_set_basis: npw Miller triples inside the grid). */
int tc_set_band_basis(tc_ctx* ctx, int ib, int npw, const int32_t* miller);

/* Orbitals of band k-point ib: nband x npw(ib) complex128 coefficients (the same nband at every band
 * k-point) and their fillings in [0, 1], which the divergence corrections of the band forms use.  All band
 * bases must be set first (TC_ERR_STATE). */
int tc_load_band_orbitals(tc_ctx* ctx, int ib, int nband, const double* coef, const double* occ);

/* Apply the two- and three-body operator of the loaded mesh orbitals (Eq. SCF with the selected terms) to
 * every band orbital: out (host, may be NULL) receives [nkb][nband][npw_max_band] complex128 (H c)(G) on
 * each band k-point's plane waves, zero-padded; eps (host, may be NULL) [nkb][nband] complex128 orbital
 * energies <phi| T + h |phi>.  The shift of each pair is k_b - k_q exactly (no reduction modulo G).  With
 * div_correction set and the correction bit selected, the band forms of the divergence corrections are
 * applied (Eqs. divcorr_2ax_band, divcorr_2bx1/2, divcorr_3a3, div_corr_3a4_2/3, div_corr_3b3_2,
 * div_corr_3b4_2/4, 3b5_div_2/3, 3b6_div_band1-3, with the band k-point's own orbitals and fillings as the
 * orbitals q_k at the singular point, and the corrections of the occupied rows' h5 of Alg. 3a2); a band
 * k-point on the mesh (modulo G) is then TC_ERR_ARG (use the mesh k-point).  TC mode, one spin channel, no
 * symmetry (TC_ERR_UNSUPPORTED otherwise). */
int tc_apply_band(tc_ctx* ctx, double* out, double* eps);

/* Crystal symmetry (Sec. 2.6.1: the orbital of k = R^T k0 - b is the image of that of k0; Sec. 2.6.4: the
 * fields h5 and h3 of the occupied-occupied pass of Algs. 3a2 and 3a4 are computed for irreducible
 * k-points only and rotated).  nsym operations x -> R (x + tau) on fractional (lattice) coordinates x:
 * rot holds nsym row-major integer 3x3 matrices R, tau nsym fractional translations.  Each operation must
 * be an isometry of the lattice, map the k-mesh onto itself and the grid onto itself (N tau integer), and
 * together they must form a group (TC_ERR_ARG otherwise).  nsym = 0 switches symmetry off.
 *
 * The representative of each k-point is the lowest k index of its orbit.  Only the representatives'
 * orbitals need to be loaded: at the next application the library replaces the orbitals and fillings
 * of every other k-point k with the image, under the first listed operation that carries its
 * representative k0 onto k, of k0's orbitals: c_k(m) = c_k0(m0) exp(2 pi i (m - b).tau) with
 * m = R^T m0 + b, so that u_k(x) = exp(2 pi i b.x) u_k0(R (x + tau)).  It checks that every
 * representative's plane-wave set and weighted occupied set are invariant under the operations that fix
 * its k-point (TC_ERR_ARG otherwise): then the operator and energy equal those of the full calculation on
 * the generated set.  The occupied-occupied pass and the target passes then run for the
 * representatives' orbitals only; the other orbitals' fields, outputs and energy contributions follow by
 * the operations.  tc_get_orbitals returns the generated orbitals after an application.
 * Built for TC mode with one spin channel (TC_ERR_UNSUPPORTED at application otherwise); tc_apply*,
 * tc_scf and tc_energy_backward* return TC_ERR_UNSUPPORTED while symmetry is set.  Call after the cell,
 * k-mesh and grid (TC_ERR_STATE otherwise); setting any of them again switches symmetry off. */
int tc_set_symmetry(tc_ctx* ctx, int nsym, const int32_t* rot, const double* tau);

/* tc_load_orbitals for spin channel `spin` (0 = up, the set of tc_load_orbitals; 1 = down, needs
 * tc_set_nspin(ctx, 2)).  left != NULL: the channel's left orbitals, biorthonormalised with its right ones
 * as in tc_load_orbitals; left orbitals must be loaded in both channels on every k-point or nowhere (else
 * TC_ERR_STATE at application).  occ are the channel's own fillings in [0, 1].  TC_ERR_STATE for spin 1
 * with one channel; TC_ERR_ARG for another spin. */
int tc_load_orbitals_spin(tc_ctx* ctx, int spin, int ik, int nband, const double* right, const double* left,
                          const double* occ);

/* Apply the selected two- and three-body terms (with corrections) to every
 * loaded orbital.  `out` (host) receives [nk][nband][npw_max] complex128
 * coefficients (H c)(G) = sqrt(Omega) FT[g](G) on each k-point's plane-wave set,
 * zero-padded to npw_max = max npw (with two spin channels, [2][nk][nband][npw_max],
 * spin-major).  The energies of this application are kept for tc_energy. */
int tc_apply_all(tc_ctx* ctx, double* out);

/* Same, writing to a caller-owned device buffer of the same layout (may be NULL:
 * the result then stays inside the context).  Asynchronous on the stream. */
int tc_apply_all_dev(tc_ctx* ctx, void* out_dev);

/* tc_apply_all_dev for callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): this call makes no hipMalloc, hipFree or other
 * allocation.  Every device buffer it needs (fields, pair buffers, partials, correction work areas, the
 * output staging) is carved from a fixed scratch array of 256 MiB that each device holds from the
 * library's load until the process ends; the context's own buffers are left as they were.  Problems
 * whose buffers do not fit, even at one target per batch, return TC_ERR_OOM (tc_set_batch can lower the
 * batch); the resident pair store is never used.  The context must have run an ordinary application
 * (tc_apply_all_dev or tc_apply_all) since its last setter or load, else TC_ERR_STATE; out_dev must not
 * be NULL (TC_ERR_ARG).  Synchronous.  All contexts on one device share its scratch, which keeps the last
 * call's contents: calls that overlap in time on one device (other threads, other streams) race. */
int tc_apply_all_dev_noalloc(tc_ctx* ctx, void* out_dev);

/* Pseudo-energy per cell (reading of Eqs. EtotTC / EtotBiTC: (1/N_k) Re sum_{sigma,k,mu}
 * f <chi| T + h2/2 + h3/3 |phi>, chi = phi in TC mode) of the last application (runs
 * one if needed).
 * e_parts: NULL or TC_E_NPARTS doubles. */
int tc_energy(tc_ctx* ctx, double* e_total, double* e_parts);

/* Apply the operator that the loaded orbitals define (h2 + h3 with the selected terms and
 * corrections, Eqs. SCF / BITCSCF, without the kinetic term) to nvec trial vectors per k-point, as
 * the block-Davidson iteration of Sec. 2.4 needs.  in and out are [nk][nvec][npw_max] complex128,
 * vector v of k-point k at (k*nvec + v); input beyond npw(k) is ignored, output beyond it is zero.
 * With two spin channels (tc_set_nspin) they are [2][nk][nvec][npw_max]: each channel's vectors
 * against that channel's operator (Eq. SCF per spin).  Every term is linear in the target: the occupied set supplies the densities, partner sums and
 * corrections, and the trial vectors take the target role (phi_j in the algorithms).  The results of
 * the last tc_apply_all* (energies, orbital energies) are not changed.  TC_ERR_ARG for nvec <= 0 or
 * null buffers. */
int tc_apply(tc_ctx* ctx, int nvec, const double* in, double* out);

/* Same, with caller-owned device buffers of the same layout.  Synchronous. */
int tc_apply_dev(tc_ctx* ctx, int nvec, const void* in_dev, void* out_dev);

/* Parameters of the self-consistent loop (Sec. 2.4). */
typedef struct {
  int max_iter;   /* iterations (one block-Davidson subspace diagonalisation each), >= 1            */
  int pmax;       /* expansion blocks per iteration: subspace of (pmax + 1) nband vectors per k,
                     0..16, at most 512 vectors                                                    */
  double etol;    /* stop when the energy per cell changes by less than etol (hartree), > 0        */
  double mix;     /* density-matrix mixing ratio beta in (0, 1]; 1 = no mixing                       */
  double otol;    /* and when no new orbital has a component above otol outside the span of the
                     previous ones (<= 0: the energy criterion alone)                               */
} tc_scf_params;

/* Block-Davidson TC-SCF (TC mode) or BITC-SCF (left orbitals loaded) from the loaded orbitals
 * (Sec. 2.4, Eq. blockDavid).  Each iteration starts the subspace with the current right orbitals
 * (orthonormalised) and adds pmax blocks of residuals (h - eps_i) v preconditioned with the function of
 * Payne et al., with Gram-Schmidt, dropping vectors of norm below 1e-8 or linearly dependent ones.  It
 * diagonalises the subspace matrix <v_a| T + h |v_b> (FP64, on the device) and takes the nband
 * eigenvectors of lowest real eigenvalue as the new orbitals: Gram-Schmidt orthonormalised in TC mode;
 * right and left eigenvectors, biorthonormalised as in tc_load_orbitals, in BITC mode.  The operator is
 * updated every iteration, with the fillings kept: built from the new orbitals, or with mix < 1 from
 * the new orbitals with fillings mix f together with the previous iteration's orbitals, as extra
 * bands, with fillings (1 - mix) f (density-matrix mixing of Sec. 2.4; the energy of an iteration is
 * that of this set).  energies (may be NULL)
 * receives the energy per cell after each iteration; iterations (may be NULL) the number run.  The
 * loop stops at max_iter, or once the energy changes by less than etol and (otol > 0) the orbitals
 * move out of their previous span by less than otol (TC energies are not stationary in the orbitals,
 * so a small energy change alone does not bound the orbitals' error).  The
 * context then holds the final orbitals alone (tc_get_orbitals) and their energies.
 * Errors: TC_ERR_ARG for parameters out of range or fewer independent trial vectors than bands;
 * TC_ERR_DEVICE if the subspace eigensolver does not converge. */
int tc_scf(tc_ctx* ctx, const tc_scf_params* prm, double* energies, int* iterations);

/* Copy the current orbitals of k-point ik to the host ([nband][npw(ik)] complex128): right (may be
 * NULL) and, in the biorthogonal mode, left (NULL, or TC_ERR_STATE without left orbitals). */
int tc_get_orbitals(tc_ctx* ctx, int ik, double* right, double* left);

/* The same for spin channel `spin` (0 or 1 with tc_set_nspin(ctx, 2)).
 * TC_ERR_ARG for a channel out of range. */
int tc_get_orbitals_spin(tc_ctx* ctx, int spin, int ik, double* right, double* left);

/* Orbital energies of the last application (runs one if needed): eps receives [nk][nband]
 * complex128, eps_j = <chi_j| T + h2 + h3 |phi_j> with the selected terms and corrections (the
 * diagonal elements of Eqs. SCF / BITCSCF, chi = phi in TC mode; Re eps_jj is the one-electron
 * energy of Sec. 2.3).  Per spin channel: one set with nspin = 1 (both channels are equal),
 * [2][nk][nband] with two channels. */
int tc_orbital_energies(tc_ctx* ctx, double* eps);

/* Gradient of the pseudo-energy of the loaded orbitals (the functional returned by
 * tc_energy, with the selected terms and corrections).  grad (host, may be NULL)
 * receives [nk][nband][npw_max] complex128 dE/dRe c + i dE/dIm c = 2 dE/dc* for the
 * coefficients shared by both spin channels, zero-padded like tc_apply_all (with two
 * channels, tc_set_nspin: [2][nk][nband][npw_max], each channel's own coefficients); dA and
 * dC (may be NULL) receive dE/dA_s and dE/dC_s (s = parallel, antiparallel) with the
 * four parameters independent.  Both are exact derivatives of the discrete energy:
 * the orbital gradient comes from one extra application whose scalar kernel is
 * 4 pi/Q^2 - (grad u)^2~ (the Hermitian part of the pair interaction of Eq. V2body,
 * whose first variation the grad-u . grad terms and their adjoints reduce to) with
 * the three-body operator of Sec. 2.6.4 unchanged; dA and dC come from energies
 * along the exact tangents of the kernel tables (Sec. 2.6.3, Appendix B) and of the
 * correction prefactors (Eqs. u_short, divcor_3a2_first/second, 3b6_div_scf1-3),
 * on which the energy depends quadratically.  Pair densities are recomputed, not
 * stored.  Cost: one application for grad, two per requested parameter.
 * Errors: TC_ERR_ARG if all three outputs are NULL; TC_ERR_UNSUPPORTED unless the
 * selected terms contain 2bh1, 2bh2, 2bx1, 2bx2 together or none of them (and then
 * also 2ah and 2ax), and all three-body terms or none.  The energies of the last
 * tc_apply_all* stay available to tc_energy; its output buffer is not. */
int tc_energy_backward(tc_ctx* ctx, double* grad, double dA[2], double dC[2]);

/* Same, writing grad to a caller-owned device buffer of the same layout (may be NULL).
 * Synchronous: returns after the stream has finished the work.  With left orbitals loaded a
 * non-NULL grad is TC_ERR_UNSUPPORTED (use tc_energy_backward_lr); dA and dC are available. */
int tc_energy_backward_dev(tc_ctx* ctx, void* grad_dev, double dA[2], double dC[2]);

/* Gradients with respect to the right and the left orbitals (host buffers, layout of
 * tc_energy_backward; each may be NULL), and dA, dC.
 *  - TC mode: grad_left must be NULL (TC_ERR_ARG); grad_right receives tc_energy_backward's gradient.
 *  - Biorthogonal mode (Eq. EtotBiTC with the biorthonormal pair held fixed; the
 *    biorthonormalisation of tc_load_orbitals is not differentiated):
 *      grad_left  = 2 dE/dchi* = 2 w (T + h) phi        (the operator of Eq. BITCSCF),
 *      grad_right = 2 dE/dphi* = 2 w (T + h^dagger) chi (the left operator of Eq. BITCSCFconj:
 *        chi and phi exchanged and v2 replaced by its adjoint, whose grad-u . grad terms change
 *        sign and whose scalar kernel becomes 4 pi/Q^2 - lap u~ - (grad u)^2~),
 *    w = f / N_k, one application each.  With two spin channels (spin-major [2][nk][nband][npw_max])
 *    each channel's gradients are those of its own pair: w (T + h) phi and w (T + h^dagger) chi.
 * Term-mask conditions and errors as tc_energy_backward. */
int tc_energy_backward_lr(tc_ctx* ctx, double* grad_right, double* grad_left, double dA[2], double dC[2]);

/* Wait for all work queued by this context. */
int tc_sync(tc_ctx* ctx);

/* Milliseconds of device time of the last tc_apply_all*, measured with events on
 * the context's stream; kernel_ms[0..n) receives the per-stage breakdown
 * (stages: 0 G->r, 1 densities and Hartree fields, 2 occupied-occupied pass,
 * 3 pass A, 4 pass B, 5 r->G and FP64 corrections).  With the resident pair store
 * (tc_set_pair_store) stage 2 includes pass A's pair densities and first z stage, and
 * with 3b6 and pass-B terms both selected stage 4 includes the shared last z stage. */
int tc_last_timing(tc_ctx* ctx, double* total_ms, double* stage_ms, int n);

/* Number of target orbitals processed per pass-A/B batch (and occupied partners per
 * batch of the occupied-occupied pass).  0 (default) sizes batches to an eighth of the
 * device's memory (between 8 and 32 GiB) of pair buffers.  Where the device cannot hold a batch's
 * pair buffers, the batch halves until it fits (down to one target).  Results do not depend on it;
 * tests use small values to cover batching. */
int tc_set_batch(tc_ctx* ctx, int targets_per_batch);

/* Resident pair store (on = 1, the default): when tc_apply_all* runs with the orbitals as targets,
 * the pass-A z-stage outputs of the orbital pairs (5 fields of N1 N2 N3 working-precision complex values
 * per pair and spin channel) are computed once, before the occupied-occupied pass, and kept.  The pair
 * (a, b) of that pass is the pass-A pair with target b and partner a (same density conj(chi_a) psi_b,
 * same momentum k_b - k_a), so the pass reads its four fields per pair from the store instead of
 * recomputing them.  TC mode keeps only the pairs (t, q) with q <= t, in triangular rows: the pair
 * (t, q) of q > t is the conjugate of (q, t)'s output at the reflected xy frequencies (its density is
 * the conjugate and its shift the negative, and every kernel is real in real space and zero on the
 * Nyquist planes).  Where not every pair fits, the store keeps the first Q1 partner columns (the pairs
 * with min(t, q) < Q1): the occupied pass forms its own pairs for its rows a >= Q1 and pass A those of
 * the targets and partners at or above Q1.  Q1 is as many columns as fit with an eighth of the
 * device's memory (at least 16 GiB) left free after the batch buffers, and none when fewer than P/8
 * fit.  The biorthogonal mode needs both orders of a pair (conj(chi_b) psi_a at k_a - k_b is the
 * pass-A pair with target a and partner b) and stores all P^2 pairs or none.  With a budget
 * (tc_set_memory_budget) the store takes what is left of it after 8 targets of pair buffers.  With on
 * = 0 both passes transform their own pair densities.  Results do not depend on it; the store is
 * released when it is switched off.  Trial vectors, band k-points and symmetry-reduced runs always
 * use the batched form. */
int tc_set_pair_store(tc_ctx* ctx, int on);

/* Kernels timed by tc_kernel_stats (device time between HIP events recorded on the
 * context's stream around every launch).  Each index names one kernel symbol of the
 * library (working precision R, grid length N), as listed by a kernel trace. */
enum {
  TC_K_SCATTER = 0,     /* k_scatter: coefficients into the FFT box                     */
  TC_K_FFT_XY_FWD = 1,  /* k_fft_xy<R,N,-1>: forward xy-plane transforms                */
  TC_K_FFT_XY_INV = 2,  /* k_fft_xy<R,N,+1>: inverse xy-plane transforms                */
  TC_K_FFT_Z_FWD = 3,   /* k_fft_z<R,N,-1>                                               */
  TC_K_FFT_Z_INV = 4,   /* k_fft_z<R,N,+1>                                               */
  TC_K_XY_PAIR_OCC = 5, /* k_pair_xy<R,N,true>: occupied-occupied pair densities, fwd xy */
  TC_K_XY_PAIR_TGT = 6, /* k_pair_xy<R,N,false>: target-partner pair densities, fwd xy  */
  TC_K_SUM_PARTS = 7,   /* k_sum_parts: fixed-order sums of the partner-chunk partials  */
  TC_K_XY_PASSB = 8,    /* k_passB_xy: pass-B sources, fwd xy                           */
  TC_K_ZCONV_OCC = 9,   /* k_zconv<R,N,OP_O>                                            */
  TC_K_ZCONV_A1 = 10,   /* k_zconv<R,N,OP_A1>                                           */
  TC_K_ZCONV_A2 = 11,   /* k_zconv<R,N,OP_A2>                                           */
  TC_K_ZCONV_B = 12,    /* k_zconv<R,N,OP_B>                                            */
  TC_K_FUSED_O = 13,    /* k_fused_O: inverse xy + partner sums, occupied-occupied pass */
  TC_K_FUSED_A = 14,    /* k_fused_A: inverse xy + partner sums of pass A, 3b6 sources  */
  TC_K_FUSED_Y = 15,    /* k_fused_Y: inverse xy + partner sums, 3b6 chain and pass B   */
  TC_K_OTHER = 16,      /* densities, Hartree-type fields, local terms, gathers          */
  TC_K_CORR = 17,       /* FP64 corrections, overlaps and kinetic energy                 */
  TC_K_FUSED_OB = 18,   /* k_fused_OB: occupied-occupied pass with left orbitals (BITC)  */
  TC_K_NKERNEL = 19
};

/* Enable (1) or disable (0) per-kernel event timing for later applications. */
int tc_set_profiling(tc_ctx* ctx, int on);

/* Accumulated device milliseconds, launch counts and algorithmic bytes (reads +
 * writes of the fields each launch must touch at least once) per kernel since
 * profiling was enabled; each array has TC_K_NKERNEL entries (NULL allowed).
 * reset != 0 clears the accumulators after reading. */
int tc_kernel_stats(tc_ctx* ctx, double* ms, double* launches, double* bytes, int reset);

#ifdef __cplusplus
}
#endif
#endif /* TCMI_H */
