// Host orchestration, FP64 set-up and corrections, and the C ABI (include/tcmi.h).
//
// One context owns one problem (cell, k-mesh, grid, basis, Jastrow parameters,
// options, orbitals) and an engine specialised on the working precision R and the
// grid length N.  An application runs, on the context's stream:
//   0  G -> r of psi = sqrt(Omega) phi and D = sqrt(Omega) (nabla + ik) phi;
//   1  densities n, J and the Hartree-type fields (Algs. 2ah, 3a1, 3b1; 2bh1/2bh2);
//   2  occupied-occupied pair pass (Algs. 3a2, 3a4 first loop, 3b2/3b5 first loop);
//   3  pass A per (target j, partner q): 2ax, 2bx1, 3a4, h4_j (Algs. 2ax, 3a3), 3b6 chain;
//   4  pass B per pair: 2bx2 + 2*(3b3 + 3b4 + 3b5) through one shared kernel -iQu;
//   5  local terms, r -> G, then the SCF-mesh divergence corrections in FP64.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <functional>
#include <list>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <type_traits>
#include <unordered_map>
#include <vector>

#include "../../include/tcmi.h"
#include "kernels.hpp"
#include "sym.hpp"
#include "band.hpp"
#include "scf.hpp"

using namespace tcmi;

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kFourPi = 4.0 * kPi;

#define TC_HIP(call)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess) {                                                              \
      throw TcError(TC_ERR_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_));   \
    }                                                                                    \
  } while (0)

struct TcError {
  int code;
  std::string msg;
  TcError(int c, std::string m) : code(c), msg(std::move(m)) {}
};

// ------------------------------------------------------------------ kernels of u = A/r (1 - e^{-r/C})
// Fourier transforms of Sec. 2.6.3 and Appendix B (non-periodic convention).
// Forward-mode derivative: value v and derivative d along one parameter (exact to rounding).
struct Dual {
  double v, d;
};
inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator/(Dual a, Dual b) { return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)}; }
inline Dual operator+(Dual a, double b) { return {a.v + b, a.d}; }
inline Dual operator+(double a, Dual b) { return {a + b.v, b.d}; }
inline Dual operator-(Dual a, double b) { return {a.v - b, a.d}; }
inline Dual operator-(double a, Dual b) { return {a - b.v, -b.d}; }
inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
inline Dual operator*(double a, Dual b) { return {a * b.v, a * b.d}; }
inline Dual operator*(Dual a, double b) { return {a.v * b, a.d * b}; }
inline Dual operator/(double a, Dual b) { return {a / b.v, -a * b.d / (b.v * b.v)}; }
inline Dual operator/(Dual a, double b) { return {a.v / b, a.d / b}; }
inline Dual atan(Dual a) { return {std::atan(a.v), a.d / (1.0 + a.v * a.v)}; }
inline double value_of(double x) { return x; }
inline double value_of(Dual x) { return x.v; }

// S is double, or Dual for derivatives with respect to A and C.
template <class S>
struct JkT {
  S u, lap, w;
};
using Jk = JkT<double>;

template <class S>
JkT<S> jastrow_ft_t(double Q2, S A, S C) {
  const S ic2 = 1.0 / (C * C);
  JkT<S> k;
  k.u = kFourPi * A * (1.0 / Q2 - 1.0 / (Q2 + ic2));
  k.lap = -kFourPi * A * ic2 / (Q2 + ic2);
  const S g = C * std::sqrt(Q2);
  S br;
  using std::atan;
  if (value_of(g) < 1e-3) {
    const S g2 = g * g;   // Taylor series of the bracket / g
    br = 0.5 - kPi * g / 4.0 + 11.0 * g2 / 24.0 - 57.0 * g2 * g2 / 480.0;
  } else {
    br = (-kPi * g * g / 4.0 - (1.0 + 0.5 * g * g) * atan(0.5 * g) + (1.0 + g * g) * atan(g)) / g;
  }
  k.w = kFourPi * A * A / C * br;
  return k;
}

inline Jk jastrow_ft(double Q2, double A, double C) { return jastrow_ft_t<double>(Q2, A, C); }

// Which kernel tables to build.
//   OPERATOR: the operator's own kernels.
//   GRADIENT: the scalar kernel V2a - L~ (L~ = -Q^2 u~, zero at Q = 0), i.e. 4 pi/Q^2 - (grad u)^2~ off
//             Q = 0 and V2a(0) at Q = 0.  With the grad-u . grad terms switched off, one application with
//             these tables gives the orbital gradient of the energy (see tc_energy_backward).
//   ADJOINT:  the scalar kernel V2a - 2 L~, i.e. 4 pi/Q^2 - L - (grad u)^2~ off Q = 0 and V2a(0) at Q = 0.
//             The discrete adjoint of the grad-u . grad terms is minus themselves minus twice the pair
//             operator with kernel L~, so the adjoint operator h^dagger is one application with these
//             tables, the grad-u . grad terms at multiplier -1 and left and right orbitals exchanged.
//   TANGENT:   every quantity that depends on (A, C) moved along its exact derivative with respect to one
//             parameter: K + h dK/dtheta (theta = A_par, A_anti, C_par, C_anti).  The energy is a
//             polynomial of degree two in these quantities taken together, so a central difference over
//             +-h along the tangent is its exact derivative.
struct TableVariant {
  enum Kind { OPERATOR = 0, GRADIENT = 1, TANGENT = 2, ADJOINT = 3 } kind = OPERATOR;
  // multiplier of L = lap u~ in the scalar kernels away from Q = 0
  double lap_factor() const { return kind == GRADIENT ? 0.0 : kind == ADJOINT ? -1.0 : 1.0; }
  int dir = 0;
  double h = 0;
};

// Quantity f(A_ch, C_ch) of spin channel ch (0 parallel, 1 antiparallel) for the variant: its value,
// plus h times its derivative (forward mode) when the variant moves a parameter of this channel.
// Tangent directions: 0 A_par, 1 A_anti, 2 C_par, 3 C_anti.
template <class F>
double chan_eval(const TableVariant& tv, const double* A, const double* C, int ch, F&& f) {
  if (tv.kind != TableVariant::TANGENT || tv.dir % 2 != ch) return f(A[ch], C[ch]);
  const Dual a{A[ch], tv.dir < 2 ? 1.0 : 0.0}, c{C[ch], tv.dir < 2 ? 0.0 : 1.0};
  const Dual v = f(a, c);
  return v.v + tv.h * v.d;
}

// u~, lap u~ and (grad u)^2~ of channel ch at Q^2 for the variant.
inline Jk chan_kernels(const TableVariant& tv, const double* A, const double* C, int ch, double Q2) {
  if (tv.kind != TableVariant::TANGENT || tv.dir % 2 != ch) return jastrow_ft(Q2, A[ch], C[ch]);
  const Dual a{A[ch], tv.dir < 2 ? 1.0 : 0.0}, c{C[ch], tv.dir < 2 ? 0.0 : 1.0};
  const JkT<Dual> k = jastrow_ft_t<Dual>(Q2, a, c);
  return Jk{k.u.v + tv.h * k.u.d, k.lap.v + tv.h * k.lap.d, k.w.v + tv.h * k.w.d};
}

// ------------------------------------------------------------------ problem description (host, FP64)
struct Problem {
  double lat[9] = {0};
  double B[9] = {0};
  double omega = 0;
  bool cell = false;
  int n1 = 0, n2 = 0, n3 = 0, nk = 0;
  int N = 0;
  std::vector<std::vector<int>> miller;   // per k, 3*npw
  std::vector<int> npw;
  int npw_max = 0;
  double A[2] = {0, 0}, C[2] = {1, 1};
  bool jastrow = false;
  int prec = TC_PREC_FP64;
  double alpha = 1.0;
  int div = 1;
  int reading = TC_DIV_PRINTED;           // TC_DIV_PRINTED or TC_DIV_LIMIT (coefficients of the mesh corrections)
  bool force_rem = false;                 // 2bx1 remainder on while the gradient application masks 2bx1 off
  uint64_t mask = TC_T_ALL;
  bool options = false;
  int nb = 0;
  std::vector<double> occ;                // [nk][nb]
  std::vector<char> loaded;               // per k
  std::vector<char> left;                 // per k: loaded with left orbitals
  bool bitc = false;                      // every k-point has left orbitals (set by prepare)
  bool negate_b = false;                  // grad-u . grad terms with sign -1 (the adjoint operator)
  int nspin = 1;                          // 2: spin-polarised, the down channel's own orbitals
  double kshift[3] = {0, 0, 0};           // Monkhorst-Pack shift of the k-mesh (mesh units)
  std::vector<double> occ_dn;             // [nk][nb] fillings of the down channel (nspin = 2)
  std::vector<char> loaded_dn;            // per k (nspin = 2)
  std::vector<char> left_dn;              // per k: the down channel loaded with left orbitals
  double delta_gb = 0, sigma_aux = 0;
  int batch = 0;                          // targets per batch (0 = automatic)
  size_t mem_budget = 0;                  // bytes for the pair store and pair buffers (0: from the device)
  int pair_store = 1;                     // keep every pair's pass-A z-stage output resident when it fits
  // crystal symmetry (tc_set_symmetry): operations x -> R (x + tau) and the k-point orbits
  int nsym = 0;
  std::vector<int> symR;                  // [nsym][9]
  std::vector<double> symT;               // [nsym][3]
  std::vector<int> krep, kop, kb;         // per k: representative, operation (-1: itself), b [3]
  std::vector<int> irr;                   // representative k-points, increasing
  bool sym_ready = false;                 // the other k-points' orbitals generated since the last load
  // band (zero-weight) k-points (tc_set_band_kpoints): fractional k, plane waves, orbitals' fillings
  int nkb = 0;
  std::vector<double> bk;                 // [nkb][3]
  std::vector<std::vector<int>> bmiller;  // per band k, 3*npw
  std::vector<int> bnpw;
  int bnb = 0;                            // orbitals per band k-point
  std::vector<double> bocc;               // [nkb][bnb]
  std::vector<char> bloaded;
  std::vector<double> bdgb, bVg;           // GB quantities per band k-point (cached for band_alpha)
  double band_alpha = -1;

  int P() const { return nk * nb; }
  long NR() const { return long(N) * N * N; }
  // k-point ik of the Monkhorst-Pack mesh: (i + s) / n per axis (s = kshift, mesh units)
  void kfrac(int ik, double* f) const {
    kfrac_mesh(ik, f);
    f[0] += kshift[0] / n1;
    f[1] += kshift[1] / n2;
    f[2] += kshift[2] / n3;
  }
  // the same without the shift: differences of mesh k-points (k - q) run over these
  void kfrac_mesh(int ik, double* f) const {
    const int i3 = ik % n3, i2 = (ik / n3) % n2, i1 = ik / (n3 * n2);
    f[0] = double(i1) / n1;
    f[1] = double(i2) / n2;
    f[2] = double(i3) / n3;
  }
};

inline int mfreq_h(int i, int N) { return i < N / 2 ? i : i - N; }

// Gygi-Baldereschi bracket of Eq. correction2 with A_aux = e^{-alpha q^2}/q^2 (Eq. aux),
// summed over the mesh and the ball exp(-alpha |k-q+G|^2) > 1e-18.  k and q are both mesh points, so
// k - q runs over the unshifted mesh whatever the shift: k = 0 and the unshifted points are used.
void gb_constant(Problem& pb) {
  const double a = pb.alpha;
  const double qmax = std::sqrt(41.45 / a);
  int mm[3];
  for (int i = 0; i < 3; ++i) {
    const double L = std::sqrt(pb.lat[3 * i] * pb.lat[3 * i] + pb.lat[3 * i + 1] * pb.lat[3 * i + 1] +
                               pb.lat[3 * i + 2] * pb.lat[3 * i + 2]);
    mm[i] = int(std::ceil(qmax * L / (2 * kPi))) + 2;
  }
  double sum = 0, comp = 0;   // Neumaier summation
  for (int ik = 0; ik < pb.nk; ++ik) {
    double f[3];
    pb.kfrac_mesh(ik, f);
    for (int m1 = -mm[0]; m1 <= mm[0]; ++m1)
      for (int m2 = -mm[1]; m2 <= mm[1]; ++m2)
        for (int m3 = -mm[2]; m3 <= mm[2]; ++m3) {
          const double c1 = m1 - f[0], c2 = m2 - f[1], c3 = m3 - f[2];
          double Q[3];
          for (int c = 0; c < 3; ++c) Q[c] = c1 * pb.B[c] + c2 * pb.B[3 + c] + c3 * pb.B[6 + c];
          const double q2 = Q[0] * Q[0] + Q[1] * Q[1] + Q[2] * Q[2];
          if (q2 <= 1e-20 || a * q2 >= 41.45) continue;
          const double t = std::exp(-a * q2) / q2;
          const double s = sum + t;
          comp += std::fabs(sum) >= std::fabs(t) ? (sum - s) + t : (t - s) + sum;
          sum = s;
        }
  }
  pb.sigma_aux = sum + comp;
  pb.delta_gb = pb.omega / (4.0 * std::sqrt(kPi * kPi * kPi * a)) - (-a + pb.sigma_aux) / pb.nk;
}

// ------------------------------------------------------------------ device buffers
// Where device memory comes from during a C-ABI call (thread-local, set by the entry point for its context):
//   t_alloc: the caller's allocator (tc_set_allocator), else hipMalloc / hipFree;
//   t_arena: the scratch of the no-allocation entry point: every allocation of the call is carved from it
//            and every release is deferred, and both are undone when the call ends (ArenaScope).
struct DevAlloc {
  void* (*alloc)(size_t bytes, void* user) = nullptr;
  void (*free)(void* p, size_t bytes, void* user) = nullptr;
  void* user = nullptr;
  hipStream_t stream = nullptr;   // the context's stream: drained before memory goes back to the caller
};
struct Arena;
thread_local const DevAlloc* t_alloc = nullptr;
thread_local Arena* t_arena = nullptr;

struct Arena {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  std::vector<std::function<void()>> undo;   // restores the buffers rebound during the call, newest first
  char* carve(size_t bytes) {
    const size_t off = (used + 255) & ~size_t(255);
    if (off + bytes > cap)
      throw TcError(TC_ERR_OOM, "the no-allocation scratch holds " + std::to_string(cap) + " bytes; this call needs more than " +
                                    std::to_string(off + bytes) + " (fewer targets per batch, tc_set_batch, may fit)");
    used = off + bytes;
    return base + off;
  }
};

template <typename T>
struct DBuf {
  T* p = nullptr;
  size_t n = 0;
  const DevAlloc* al = nullptr;   // the allocator that made p (null: hipMalloc)
  bool carved = false;            // p lies in the no-allocation scratch
  void remember() {               // under an arena: the state to restore when the call ends
    t_arena->undo.push_back([this, p0 = p, n0 = n, al0 = al, c0 = carved] {
      p = p0;
      n = n0;
      al = al0;
      carved = c0;
    });
  }
  void alloc(size_t count) {
    if (t_arena) {   // rebind to the scratch (a buffer carved earlier in this call is reused when large enough)
      if (carved && count <= n) return;
      remember();
      p = count ? reinterpret_cast<T*>(t_arena->carve(count * sizeof(T))) : nullptr;
      n = count;
      al = nullptr;
      carved = true;
      return;
    }
    if (count <= n && p) return;
    release();
    if (count == 0) return;
    if (t_alloc && t_alloc->alloc) {
      p = static_cast<T*>(t_alloc->alloc(count * sizeof(T), t_alloc->user));
      if (!p) throw TcError(TC_ERR_OOM, "the caller's allocator returned NULL for " + std::to_string(count * sizeof(T)) + " bytes");
      al = t_alloc;
    } else {
      hipError_t e = hipMalloc(&p, count * sizeof(T));
      if (e != hipSuccess) {
        p = nullptr;
        (void)hipGetLastError();   // the failure is reported here, not to the caller's next launch check
        throw TcError(TC_ERR_OOM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed");
      }
      al = nullptr;
    }
    n = count;
  }
  void release() {
    if (t_arena) {   // no free inside the no-allocation call: hide the buffer until the call ends
      if (!p) return;
      if (!carved) remember();
      p = nullptr;
      n = 0;
      carved = false;
      return;
    }
    if (p && !carved) {
      if (al) {
        (void)hipStreamSynchronize(al->stream);   // no queued kernel may still use the memory
        al->free(p, n * sizeof(T), al->user);
      } else {
        (void)hipFree(p);
      }
    }
    p = nullptr;
    n = 0;
    al = nullptr;
    carved = false;
  }
  ~DBuf() { release(); }
};

struct Shared {                       // precision-independent device data
  DBuf<double> coef;                  // [P][npw_max] complex128
  DBuf<double> coefL;                 // [P][npw_max] complex128 left orbitals (biorthogonal mode)
  DBuf<double> bo_l, bo_s, bo_inv, bo_aug;   // biorthogonalisation of one k-point (FP64)
  DBuf<int> bo_flag;
  DBuf<int> boxidx;                   // [nk][npw_max]
  DBuf<int> npw;                      // [nk]
  DBuf<double> kg;                    // [nk][npw_max][3]
  DBuf<double> w;                     // [P]  f / N_k
  DBuf<double> dfr;                   // [nDelta][3]
  DBuf<double> out;                   // [P][npw_max] complex128 (H c)
  DBuf<double> grad;                  // [P][npw_max] complex128 energy gradient
  DBuf<double> dhc2, dhc3;            // FP64 corrections
  DBuf<double> epart;                 // [P][kAccSlots]
  DBuf<double> tkin;                  // [P]
  DBuf<double> S;                     // [nk][nb][nb] complex overlaps
  DBuf<double> O;                     // [nk][nb][nb] complex <c_mu | Z_j>
  DBuf<double> Zg, Wg;                // [P][npw_max] complex
  DBuf<double> ecorr;                 // [P][2]
  DBuf<double> eps;                   // [P] complex orbital energies
  // target-set side of the corrections (tc_apply)
  DBuf<double> ZgT, WgT, dhc2T, dhc3T, ST, OT, ecorrT;
  // symmetry expansion: per-k operation data, representatives, coefficient maps, and the outputs and
  // energy slots of the representatives' orbitals
  DBuf<SymK> symk;
  DBuf<int> irrk, symg0;                // [nirr], [nk][npw_max]
  DBuf<double> symph;                   // [nk][npw_max] complex phases
  DBuf<double> outI, epartI;            // [nirr nb][npw_max] complex, [nirr nb][kAccSlots]
  // band k-points: coefficients [nkb][bnb][bnpm] (complex128), plane-wave data, k codes, output, energies
  DBuf<double> bcoef, bkg, bout, beps;
  DBuf<double> bdh4, bV, bOBh4, bOB3, bZ5, bOB6, bW4, bX6, bWa;   // band corrections
  DBuf<int> bbox, bnpwd, btk;
  int bnpm = 0;
};

// ------------------------------------------------------------------ FP64 helper kernels
__global__ void k_overlap(const double* a, int na, const double* b, int nbb, const int* npw, int npw_max, int nk,
                          double* S) {
  // S[k][m][n] = sum_g conj(a_km[g]) b_kn[g], m < na (rows of a per k), n < nbb (rows of b per k)
  const int id = blockIdx.x;
  const int k = id / (na * nbb), m = (id / nbb) % na, n = id % nbb;
  const double* x = a + 2 * (long(k * na + m) * npw_max);
  const double* y = b + 2 * (long(k * nbb + n) * npw_max);
  double sr = 0, si = 0;
  for (int g = threadIdx.x; g < npw[k]; g += blockDim.x) {
    sr += x[2 * g] * y[2 * g] + x[2 * g + 1] * y[2 * g + 1];
    si += x[2 * g] * y[2 * g + 1] - x[2 * g + 1] * y[2 * g];
  }
  wg_sum2(sr, si);
  if (threadIdx.x == 0) {
    S[2 * id] = sr;
    S[2 * id + 1] = si;
  }
}

// t[p] = Re <chi_p| -lap/2 |psi_p> from the coefficients (Sec. 2.6.2); cl = c in TC mode
__global__ void k_kinetic(const double* cl, const double* c, const double* kg, const int* npw, int nb, int npw_max,
                          double* t) {
  const int p = blockIdx.x, k = p / nb;
  double s = 0;
  for (int g = threadIdx.x; g < npw[k]; g += blockDim.x) {
    const double* q = kg + (long(k) * npw_max + g) * 3;
    const double e = 0.5 * (q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
    const double* x = cl + 2 * (long(p) * npw_max + g);
    const double* y = c + 2 * (long(p) * npw_max + g);
    s += e * (x[0] * y[0] + x[1] * y[1]);
  }
  s = wg_sum(s);
  if (threadIdx.x == 0) t[p] = s;
}

// Orbital gradient from an application: grad_p = scale w_p [(h' c_p)(G) + |k+G|^2/2 c_p(G)], w_p = f_p / N_k.
// TC mode: scale 4 (both spin channels share c, and bra and ket), h' with the GRADIENT tables and the
// grad-u . grad terms off.  Biorthogonal mode: scale 2 for each of the right and left gradients.
__global__ void k_grad_finish(const double* c, const double* out, const double* kg, const int* npw, const double* w,
                              int nb, int npw_max, int P, double scale, double* grad) {
  const long id = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id >= long(P) * npw_max) return;
  const int p = int(id / npw_max), g = int(id - long(p) * npw_max), k = p / nb;
  double* o = grad + 2 * id;
  if (g >= npw[k]) {
    o[0] = o[1] = 0.0;
    return;
  }
  const double* q = kg + (long(k) * npw_max + g) * 3;
  const double e = 0.5 * (q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
  const double f = scale * w[p];
  o[0] = f * (out[2 * id] + e * c[2 * id]);
  o[1] = f * (out[2 * id + 1] + e * c[2 * id + 1]);
}

// eps[j] = <chi_j| T + h |phi_j> = sum_G conj(cl_j) [(h c)_j + |k+G|^2/2 c_j]   (complex, one block per orbital;
// cl = c in TC mode).  The bracket over the plane-wave set equals the one over the grid: chi_j has no
// components outside it.
__global__ void __launch_bounds__(256) k_orbital_eps(const double* cl, const double* c, const double* hc,
                                                     const double* kg, const int* npw, int nb, int npw_max,
                                                     double* eps) {
  const int j = blockIdx.x, k = j / nb;
  double sr = 0, si = 0;
  for (int g = threadIdx.x; g < npw[k]; g += blockDim.x) {
    const double* q = kg + (long(k) * npw_max + g) * 3;
    const double e = 0.5 * (q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
    const long o = 2 * (long(j) * npw_max + g);
    const double yr = hc[o] + e * c[o], yi = hc[o + 1] + e * c[o + 1];
    sr += cl[o] * yr + cl[o + 1] * yi;
    si += cl[o] * yi - cl[o + 1] * yr;
  }
  wg_sum2(sr, si);
  if (threadIdx.x == 0) {
    eps[2 * j] = sr;
    eps[2 * j + 1] = si;
  }
}

// ------------------------------------------------------------------ biorthogonalisation (FP64)
// Sec. 2.3 (BITC): the left and right determinants are built from orbitals with <chi_i|phi_j> = delta_ij
// and <phi_i|phi_i> = 1.  Per k-point each right orbital is normalised, S_ij = <chi_i|phi_j> is formed and
// the left set becomes conj(S^-1) chi, for which <chi'_i|phi_j> = sum_m (S^-1)_im S_mj = delta_ij.

// c_b <- c_b / ||c_b|| for the bands at c (one block per band); bad = 1 for a zero orbital
__global__ void __launch_bounds__(256) k_bo_normalize(double* c, int npw, int npw_max, int* bad) {
  double* x = c + 2 * long(blockIdx.x) * npw_max;
  double s = 0;
  for (int g = threadIdx.x; g < npw; g += blockDim.x) s += x[2 * g] * x[2 * g] + x[2 * g + 1] * x[2 * g + 1];
  s = wg_sum(s);
  const double nrm = sqrt(s);
  if (!(nrm > 0.0)) {
    if (threadIdx.x == 0) bad[0] = 1;
    return;
  }
  for (int g = threadIdx.x; g < npw; g += blockDim.x) {
    x[2 * g] /= nrm;
    x[2 * g + 1] /= nrm;
  }
}

// Sinv = S^-1 of one nb x nb complex matrix (row-major, interleaved) by Gauss-Jordan elimination with
// partial pivoting, one work-group; a: scratch of nb x 2nb + nb complex.  bad = 2 when a pivot is not
// above 1e-13 max|S_ij| (singular overlap); Sinv is then left unwritten.
__global__ void __launch_bounds__(256) k_bo_invert(const double* S, int nb, double* a, double* Sinv, int* bad) {
  const int tid = threadIdx.x, nt = blockDim.x, W = 2 * nb;
  double* fac = a + 2L * nb * W;   // column of elimination factors
  __shared__ double smax;
  __shared__ int piv, fail;
  for (long e = tid; e < long(nb) * W; e += nt) {
    const int i = int(e / W), j = int(e % W);
    a[2 * e] = j < nb ? S[2 * (long(i) * nb + j)] : (j - nb == i ? 1.0 : 0.0);
    a[2 * e + 1] = j < nb ? S[2 * (long(i) * nb + j) + 1] : 0.0;
  }
  if (tid == 0) {
    double m = 0;
    for (long e = 0; e < long(nb) * nb; ++e) m = fmax(m, hypot(S[2 * e], S[2 * e + 1]));
    smax = m;
    fail = !(m > 0.0);
  }
  __syncthreads();
  for (int k = 0; k < nb && !fail; ++k) {
    if (tid == 0) {
      int p = k;
      double best = -1.0;
      for (int i = k; i < nb; ++i) {
        const double v = hypot(a[2 * (long(i) * W + k)], a[2 * (long(i) * W + k) + 1]);
        if (v > best) {
          best = v;
          p = i;
        }
      }
      piv = p;
      if (!(best > 1e-13 * smax)) fail = 1;
    }
    __syncthreads();
    if (fail) break;
    if (piv != k)
      for (int j = tid; j < W; j += nt)
        for (int c = 0; c < 2; ++c) {
          const double t = a[2 * (long(k) * W + j) + c];
          a[2 * (long(k) * W + j) + c] = a[2 * (long(piv) * W + j) + c];
          a[2 * (long(piv) * W + j) + c] = t;
        }
    __syncthreads();
    const double pr = a[2 * (long(k) * W + k)], pi = a[2 * (long(k) * W + k) + 1];
    const double d = pr * pr + pi * pi, ir = pr / d, ii = -pi / d;
    __syncthreads();
    for (int j = tid; j < W; j += nt) {
      const double xr = a[2 * (long(k) * W + j)], xi = a[2 * (long(k) * W + j) + 1];
      a[2 * (long(k) * W + j)] = xr * ir - xi * ii;
      a[2 * (long(k) * W + j) + 1] = xr * ii + xi * ir;
    }
    for (int i = tid; i < nb; i += nt) {
      fac[2 * i] = a[2 * (long(i) * W + k)];
      fac[2 * i + 1] = a[2 * (long(i) * W + k) + 1];
    }
    __syncthreads();
    for (long e = tid; e < long(nb) * W; e += nt) {
      const int i = int(e / W), j = int(e % W);
      if (i == k) continue;
      const double fr = fac[2 * i], fi = fac[2 * i + 1];
      const double yr = a[2 * (long(k) * W + j)], yi = a[2 * (long(k) * W + j) + 1];
      a[2 * e] -= fr * yr - fi * yi;
      a[2 * e + 1] -= fr * yi + fi * yr;
    }
    __syncthreads();
  }
  if (fail) {
    if (tid == 0 && bad[0] == 0) bad[0] = 2;   // a zero right orbital (1) is the more specific report
    return;
  }
  for (long e = tid; e < long(nb) * nb; e += nt) {
    const int i = int(e / nb), j = int(e % nb);
    Sinv[2 * e] = a[2 * (long(i) * W + nb + j)];
    Sinv[2 * e + 1] = a[2 * (long(i) * W + nb + j) + 1];
  }
}

// out_i = sum_m conj(Sinv_im) l_m for the nb bands of one k-point ([nb][npw_max], zero beyond npw)
__global__ void k_bo_left(const double* Sinv, const double* l, int nb, int npw, int npw_max, double* out) {
  const long id = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id >= long(nb) * npw_max) return;
  const int i = int(id / npw_max), g = int(id - long(i) * npw_max);
  double re = 0, im = 0;
  if (g < npw)
    for (int m = 0; m < nb; ++m) {
      const double sr = Sinv[2 * (long(i) * nb + m)], si = Sinv[2 * (long(i) * nb + m) + 1];
      const double xr = l[2 * (long(m) * npw_max + g)], xi = l[2 * (long(m) * npw_max + g) + 1];
      re += sr * xr + si * xi;
      im += sr * xi - si * xr;
    }
  out[2 * id] = re;
  out[2 * id + 1] = im;
}

// Source of the G != 0 correction of 3a2 (Eq. divcor_3a2_second, general-overlap form):
// Y = 2 sum_k sum_{m1,m2} (f_m1 f_m2 / N_k) (S(m1,m2)/Omega) conj(chi_m2) psi_m1, S(a,b) = <chi_a|psi_b>
template <int N>
__global__ void k_corr_Ysrc(const cx<double>* chi, const cx<double>* psi, const double* S, const double* f, int nk,
                            int nb, double inv_nk_omega, cx<double>* Y) {
  constexpr long NR = long(N) * N * N;
  const long r = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= NR) return;
  double yr = 0, yi = 0;
  for (int k = 0; k < nk; ++k)
    for (int m1 = 0; m1 < nb; ++m1)
      for (int m2 = 0; m2 < nb; ++m2) {
        const int i1 = k * nb + m1, i2 = k * nb + m2;
        const double sr = S[2 * ((k * nb + m1) * nb + m2)], si = S[2 * ((k * nb + m1) * nb + m2) + 1];
        const cx<double> v = cmulc(chi[i2 * NR + r], psi[i1 * NR + r]);
        const double c = 2.0 * f[i1] * f[i2] * inv_nk_omega;
        yr += c * (sr * v.x - si * v.y);
        yi += c * (sr * v.y + si * v.x);
      }
  Y[r] = {yr, yi};
}

// G-space fields of the corrections: F3b6~ = sum_s (2 pi A_s / N_k) u_s n~, F2~ = sum_s (4 pi A_s / N_k) u_s Y~
template <int N>
__global__ void k_corr_gfields(const double* u0, const double* u1, double c0, double c1, const cx<double>* in,
                               cx<double>* out) {
  constexpr long NR = long(N) * N * N;
  const long r = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= NR) return;
  out[r] = (c0 * u0[r] + c1 * u1[r]) * in[r];
}

// spin-polarised form: out = c0 u0 in_own + c1 u1 in_other
template <int N>
__global__ void k_corr_gfields2(const double* u0, const double* u1, double c0, double c1, const cx<double>* in,
                                const cx<double>* ino, cx<double>* out) {
  constexpr long NR = long(N) * N * N;
  const long r = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= NR) return;
  out[r] = (c0 * u0[r]) * in[r] + (c1 * u1[r]) * ino[r];
}

// per-orbital products F * psi_p for two fields (batched output [2][P][NR])
template <int N>
__global__ void k_corr_products(const cx<double>* F, const cx<double>* psi, int P, cx<double>* out) {
  constexpr long NR = long(N) * N * N;
  const long id = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id >= 2L * P * NR) return;
  const long fi = id / (long(P) * NR);
  const long rem = id - fi * long(P) * NR;
  const long p = rem / NR, r = rem - p * NR;
  out[id] = F[fi * NR + r] * psi[p * NR + r];
}

// corrections in coefficient space (FP64), S(a,b) = <chi_a|psi_b>, O(a,b) = <chi_a|F psi_b>:
//  dhc2_j = -4 pi dGB sum_mu f_mu (S(mu,j)/Omega) c_mu                        (Eq. divcorr_2ax_scf)
//  dhc3_j = 1/2 const1 c_j + 1/2 W_j                                          (3a2, Eqs. divcor_3a2_*)
//         + 2 sum_mu f_mu { [c1s n0 S(mu,j)/Omega + O(mu,j)/Omega] c_mu + (S(mu,j)/Omega) Z_mu }  (3b6 x 2)
// const1 and c1s n0 are complex (imaginary parts zero in TC mode).
// Targets j (coefficients cT, nbt per k-point) may differ from the occupied set c (nb per k-point);
// S and O are then [k][mu][jb] with rows of length nbt, and W is per target.
__global__ void k_corr_apply(const double* cT, const double* c, const double* S, const double* O, const double* Z,
                             const double* W, const double* f, const int* npw, int nb, int nbt, int npw_max, int NT,
                             double omega, double m2ax, double dgb, double m3a2, double const1, double const1i,
                             double m3b6, double c1s_n0, double c1s_n0i, double* dhc2, double* dhc3) {
  const long id = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id >= long(NT) * npw_max) return;
  const int j = int(id / npw_max), g = int(id - long(j) * npw_max);
  const int k = j / nbt, jb = j % nbt;
  double a2r = 0, a2i = 0, a3r = 0, a3i = 0;
  if (g < npw[k]) {
    const double* cj = cT + 2 * (long(j) * npw_max + g);
    for (int mu = 0; mu < nb; ++mu) {
      const int q = k * nb + mu;
      const double* cq = c + 2 * (long(q) * npw_max + g);
      const double* zq = Z + 2 * (long(q) * npw_max + g);
      const long si = 2 * ((long(k) * nb + mu) * nbt + jb);
      const double sr = S[si] / omega, sim = S[si + 1] / omega;
      const double orr = O[si] / omega, oi = O[si + 1] / omega;
      // 2ax
      a2r += -kFourPi * dgb * f[q] * (sr * cq[0] - sim * cq[1]);
      a2i += -kFourPi * dgb * f[q] * (sr * cq[1] + sim * cq[0]);
      // 3b6 (x 2)
      const double br = c1s_n0 * sr - c1s_n0i * sim + orr, bi = c1s_n0 * sim + c1s_n0i * sr + oi;
      a3r += 2.0 * m3b6 * f[q] * (br * cq[0] - bi * cq[1] + sr * zq[0] - sim * zq[1]);
      a3i += 2.0 * m3b6 * f[q] * (br * cq[1] + bi * cq[0] + sr * zq[1] + sim * zq[0]);
    }
    const double* wj = W + 2 * (long(j) * npw_max + g);
    a3r += m3a2 * 0.5 * (const1 * cj[0] - const1i * cj[1] + wj[0]);
    a3i += m3a2 * 0.5 * (const1 * cj[1] + const1i * cj[0] + wj[1]);
  }
  dhc2[2 * id] = m2ax * a2r;
  dhc2[2 * id + 1] = m2ax * a2i;
  dhc3[2 * id] = a3r;
  dhc3[2 * id + 1] = a3i;
}

// out += dhc2 + dhc3;  ecorr[j] = (<cl_j|dhc2_j>, <cl_j|dhc3_j>) real parts (cl: left coefficients, c in TC mode)
__global__ void k_corr_add(const double* c, const double* dhc2, const double* dhc3, const int* npw, int nb,
                           int npw_max, double* out, double* ecorr) {
  const int j = blockIdx.x, k = j / nb;
  double e2 = 0, e3 = 0;
  for (int g = threadIdx.x; g < npw_max; g += blockDim.x) {
    const long o = 2 * (long(j) * npw_max + g);
    if (g < npw[k]) {
      e2 += c[o] * dhc2[o] + c[o + 1] * dhc2[o + 1];
      e3 += c[o] * dhc3[o] + c[o + 1] * dhc3[o + 1];
      out[o] += dhc2[o] + dhc3[o];
      out[o + 1] += dhc2[o + 1] + dhc3[o + 1];
    }
  }
  wg_sum2(e2, e3);
  if (threadIdx.x == 0) {
    ecorr[2 * j] = e2;
    ecorr[2 * j + 1] = e3;
  }
}


// density only (FP64 corrections): n = sum_q w_q conj(chi_q) psi_q (chi = psi in TC mode)
template <int N>
__global__ void k_density64(const cx<double>* chi, const cx<double>* psi, const double* w, int P, cx<double>* n) {
  constexpr long NR = long(N) * N * N;
  const long r = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= NR) return;
  double s = 0, si = 0;
  if (chi == psi) {
    for (int q = 0; q < P; ++q) {
      const cx<double> a = psi[q * NR + r];
      s += w[q] * (a.x * a.x + a.y * a.y);
    }
  } else {
    for (int q = 0; q < P; ++q) {
      const cx<double> v = cmulc(chi[q * NR + r], psi[q * NR + r]);
      s += w[q] * v.x;
      si += w[q] * v.y;
    }
  }
  n[r] = {s, si};
}

inline unsigned nblk(long n, int b = 256) { return unsigned((n + b - 1) / b); }

// ------------------------------------------------------------------ per-family event timing
struct Prof {
  bool on = false;
  double ms[TC_K_NKERNEL] = {0}, launches[TC_K_NKERNEL] = {0}, bytes[TC_K_NKERNEL] = {0};
  struct Rec {
    int fam;
    hipEvent_t a, b;
    double bytes;
  };
  std::vector<hipEvent_t> pool;
  size_t used = 0;
  std::vector<Rec> recs;
  hipEvent_t get() {
    if (used == pool.size()) {
      hipEvent_t e;
      TC_HIP(hipEventCreate(&e));
      pool.push_back(e);
    }
    return pool[used++];
  }
  // call after the stream has been synchronised
  void collect() {
    for (const Rec& r : recs) {
      float t = 0;
      TC_HIP(hipEventElapsedTime(&t, r.a, r.b));
      ms[r.fam] += t;
      launches[r.fam] += 1;
      bytes[r.fam] += r.bytes;
    }
    recs.clear();
    used = 0;
  }
  void reset() {
    for (int i = 0; i < TC_K_NKERNEL; ++i) ms[i] = launches[i] = bytes[i] = 0;
  }
  ~Prof() {
    for (auto e : pool) (void)hipEventDestroy(e);
  }
};

struct ProfScope {
  Prof* p;
  hipStream_t s;
  int fam;
  double bytes;
  hipEvent_t a = nullptr;
  ProfScope(Prof* p_, hipStream_t s_, int f, double b) : p(p_), s(s_), fam(f), bytes(b) {
    if (p && p->on) {
      a = p->get();
      TC_HIP(hipEventRecord(a, s));
    }
  }
  ~ProfScope() noexcept(false) {
    if (p && p->on) {
      hipEvent_t b = p->get();
      TC_HIP(hipEventRecord(b, s));
      p->recs.push_back({fam, a, b, bytes});
    }
  }
};

template <typename R, int N>
void fft3d_t(cx<R>* d, long nvol, int dir, hipStream_t s, Prof* pf = nullptr) {
  if (nvol <= 0) return;
  constexpr int PB = XY<R, N>::PB;
  const long np = nvol * N;
  const double by = 2.0 * double(sizeof(cx<R>)) * nvol * N * N * N;
  if (dir < 0) {
    {
      ProfScope ps(pf, s, TC_K_FFT_XY_FWD, by);
      hipLaunchKernelGGL((k_fft_xy<R, N, -1>), dim3(nblk(np, PB)), dim3(PB * N), 0, s, d, np);
    }
    ProfScope ps(pf, s, TC_K_FFT_Z_FWD, by);
    hipLaunchKernelGGL((k_fft_z<R, N, -1>), dim3(nblk(nvol * N * N)), dim3(256), 0, s, d, nvol);
  } else {
    {
      ProfScope ps(pf, s, TC_K_FFT_Z_INV, by);
      hipLaunchKernelGGL((k_fft_z<R, N, 1>), dim3(nblk(nvol * N * N)), dim3(256), 0, s, d, nvol);
    }
    ProfScope ps(pf, s, TC_K_FFT_XY_INV, by);
    hipLaunchKernelGGL((k_fft_xy<R, N, 1>), dim3(nblk(np, PB)), dim3(PB * N), 0, s, d, np);
  }
}

// ------------------------------------------------------------------ engine
// Trial vectors of tc_apply: nvec per k-point, device coefficients [nk][nvec][npw_max] (complex128), and the
// output of the same layout.  Without a target set the targets are the loaded orbitals themselves.
struct TargetSet {
  const double* coef = nullptr;
  int nvec = 0;
  double* out = nullptr;
  // band targets (tc_apply_band): nblk k-points coded tk[] = nk + b, with their own plane-wave data
  int nblk = 0;                         // 0: one block per mesh k-point
  const int* tk = nullptr;
  const int* boxidx = nullptr;
  const int* npw = nullptr;
  const double* kg = nullptr;
  int npm = 0;
  bool band = false;
  // band divergence corrections (null: off): device a-coefficients of the h4 correction [NTG][nvec]
  // complex, V of each band k-point [nblk][3], and the outputs of the grid pieces
  const double* bdh4 = nullptr;
  const double* bV = nullptr;
  double* OBh4 = nullptr;   // [NTG][nvec][3] complex: <psi_mu | h4_j> / N^3 (corrected h4)
  double* OB3 = nullptr;    // [NTG][nvec][3] complex: <psi_mu | psi_j h1_c> / N^3
  double* Z5 = nullptr;     // [NTG][nvec][3] complex: <H3B_mu,c | psi_j> / N^3 (H3 of the band rows)
  double* OB6 = nullptr;    // [NTG][nvec] complex: <psi_mu | F3b6 psi_j> / N^3
  double* W4 = nullptr;     // [NTG][npm] complex: (V . H3B_j)(G) on the band plane waves
  double* X6 = nullptr;     // [NTG][npm] complex: (F3b6 psi_j)(G)
  double* Wa = nullptr;     // [NTG][npm] complex: (F2 psi_j)(G), the 3a2 field of the occupied set
  double c3b6[2] = {0, 0};  // -2 pi A_ch, the 3b6 band-field prefactors per channel
};

struct Engine {
  virtual ~Engine() = default;
  virtual void upload_tables(const Problem& pb, const TableVariant& tv) = 0;
  virtual void apply(hipStream_t s, Shared& sh, const Problem& pb, double* stage_ms,
                     const TargetSet* ts = nullptr) = 0;
  virtual void release_pair_store() = 0;
  Prof* prof = nullptr;
};



Masks make_masks(uint64_t m) {
  auto b = [&](uint64_t bit) { return (m & bit) ? 1.0 : 0.0; };
  Masks k;
  k.m2ah = b(TC_T_2AH); k.m2bh1 = b(TC_T_2BH1); k.m2bh2 = b(TC_T_2BH2);
  k.m2ax = b(TC_T_2AX); k.m2bx1 = b(TC_T_2BX1); k.m2bx2 = b(TC_T_2BX2);
  k.m3a1 = b(TC_T_3A1); k.m3a2 = b(TC_T_3A2); k.m3a3 = b(TC_T_3A3); k.m3a4 = b(TC_T_3A4);
  k.m3b1 = b(TC_T_3B1); k.m3b2 = b(TC_T_3B2); k.m3b3 = b(TC_T_3B3); k.m3b4 = b(TC_T_3B4);
  k.m3b5 = b(TC_T_3B5); k.m3b6 = b(TC_T_3B6);
  return k;
}

// Reading TC_DIV_LIMIT: whether the mesh targets get the 2bx1 remainder (selected 2bx1, or the gradient
// application, which masks the grad-u . grad convolutions off but keeps every Hermitian correction).
inline bool rem_2bx1(const Problem& pb) {
  return pb.reading == TC_DIV_LIMIT && ((pb.mask & TC_T_2BX1) || pb.force_rem);
}

// 2ax correction bracket and 2bx1 remainder in one coefficient: both are -4 pi c sum_mu f rho~_{mu j}(0) phi_mu
// (Eq. divcorr_2ax_scf with c = Delta_GB; the remainder with c = A_par / N_k).
inline double dgb_eff(const Problem& pb, const Masks& m, double a_par) {
  return m.m2ax * pb.delta_gb + (rem_2bx1(pb) ? a_par / pb.nk : 0.0);
}

inline bool need_corr(const Problem& pb, const Masks& m) {
  return pb.div && (pb.mask & TC_T_CORR) && (m.m2ax || m.m3a2 || m.m3b6 || rem_2bx1(pb));
}

// Stage-timing events of one application.  The no-allocation entry point creates none (its stage times
// read 0): rec() and ms() then do nothing and sync() waits on the stream.
struct Events {
  std::vector<hipEvent_t> e;
  explicit Events(int n) : e(t_arena ? 0 : n, nullptr) {
    for (auto& x : e) TC_HIP(hipEventCreate(&x));
  }
  ~Events() {
    for (auto& x : e)
      if (x) (void)hipEventDestroy(x);
  }
  void rec(int i, hipStream_t s) {
    if (i < int(e.size())) TC_HIP(hipEventRecord(e[i], s));
  }
  void sync(int i, hipStream_t s) {
    if (i < int(e.size()))
      TC_HIP(hipEventSynchronize(e[i]));
    else
      TC_HIP(hipStreamSynchronize(s));
  }
  float ms(int a, int b) const {
    if (e.empty()) return 0.f;
    float t = 0;
    TC_HIP(hipEventElapsedTime(&t, e[a], e[b]));
    return t;
  }
};

template <typename R, int N>
struct EngineT : Engine {
  static constexpr long NR = long(N) * N * N;
  static constexpr int PB = XY<R, N>::PB;
  static constexpr int NTH = Fz<R, N>::NTH;
  // working-precision fields
  DBuf<cx<R>> psi;     // [P][NR]
  DBuf<cx<R>> D;       // [3][P][NR]
  DBuf<cx<R>> Dl;      // [3][P][NR]  lattice components B D
  DBuf<cx<R>> Hl;      // [P][3][NR]  lattice components B H3a4
  DBuf<cx<R>> nJ;      // [4][NR]  n, J_x, J_y, J_z
  DBuf<cx<R>> loc;     // [8][NR]  VH, h1 x3, P2bh2, F3b1, h6, F3b2
  DBuf<cx<R>> wk;      // [9][NR]  scratch volumes
  DBuf<cx<R>> H3a4;    // [P][3][NR]
  DBuf<R> h5;          // [P][NR]
  DBuf<cx<R>> bufA;    // [T*P][4][NR]  pair densities, 3b6 and pass-B sources
  DBuf<cx<R>> bufB;    // [T*P][5][NR]  z-stage outputs; after pass A, pass-B sources and the shared z-stage output
  DBuf<cx<R>> allB;    // [P*P][5][NR]  pass-A z-stage outputs of every pair (resident store)
  DBuf<cx<R>> h4, Z;   // [T][3][NR]  h4 (Cartesian), pass-B target factor (lattice)
  DBuf<cx<R>> g;       // [T][NR]
  DBuf<cx<double>> acc;     // [kAccSlots][T][NR]  FP64 accumulation of the operator output, per energy slot
  DBuf<cx<R>> gpart;        // [S][T][3][NR]  partner-chunk partials
  DBuf<cx<R>> h4part;       // [S][T][3][NR]
  DBuf<R> h5part;           // [S][T][NR]
  DBuf<cx<R>> H3part;       // [S][T][3][NR]
  // biorthogonal mode (left orbitals chi != psi)
  DBuf<cx<R>> chi;          // [P][NR]
  DBuf<cx<R>> H3bc;         // [P][3][NR]  conj(H3b) (Cartesian), then its lattice components B conj(H3b)
  DBuf<cx<R>> h5c;          // [P][NR]  complex h5
  DBuf<cx<R>> h5cpart;      // [S][T][NR]
  DBuf<cx<R>> Hbpart;       // [S][T][3][NR]
  DBuf<cx<double>> chi64;   // [P][NR]  FP64 left orbitals for the corrections
  bool bitc_alloc = false;
  // spin-polarised runs: the down channel's fields, the antiparallel-channel h5 of each channel, scratch
  DBuf<cx<R>> psi1, D1, Dl1, Hl1, H3a4_1, nJ1, loc1, wk2;
  DBuf<R> h5_1, h5a0, h5a1;
  DBuf<cx<double>> psi64_1, v64p;
  // spin-polarised biorthogonal mode: the down channel's left fields and conj(H3b), the complex h5 of each
  // channel (the up channel's parallel part is h5c)
  DBuf<cx<R>> chi1, H3bc_1, h5c_1, h5ca0, h5ca1;
  DBuf<cx<double>> chi64_1;
  int nspin_alloc = 1;
  // target set of tc_apply (trial vectors)
  DBuf<cx<R>> psiT, DT;              // [NT][NR], [3][NT][NR]
  DBuf<cx<R>> H3I;                   // [nirr nb][3][NR]  H3a4 of the representatives' orbitals
  DBuf<R> h5I;                       // [nirr nb][NR]
  DBuf<cx<double>> psiT64, prodT;    // [NT][NR], [2][NT][NR]
  int S = 1;
  // kernel tables (scaled by 1/(Omega N^3))
  DBuf<R> tV, tU1, tU2, tHV, tHU;
  DBuf<R> tHVp, tHVa, tHUp, tHUa;   // Hartree tables per channel (spin-polarised runs)
  DBuf<double> dfr;
  // FP64 side of the corrections
  DBuf<cx<double>> psi64, v64, prod64;
  DBuf<double> tHu0, tHu1, focc;
  double corrA[2] = {0, 0}, corrB[2] = {0, 0};
  int T = 1;
  int P_alloc = -1;
  int batch_alloc = -1;

  static bool grid_q(const Problem& pb, long r, const double* f, double* Q, double& q2) {
    const int x = int(r % N), y = int((r / N) % N), z = int(r / (N * N));
    const int m1 = mfreq_h(x, N), m2 = mfreq_h(y, N), m3 = mfreq_h(z, N);
    if (m1 == -N / 2 || m2 == -N / 2 || m3 == -N / 2) return false;   // Nyquist planes carry no kernel
    const double c1 = (f ? f[0] : 0) + m1, c2 = (f ? f[1] : 0) + m2, c3 = (f ? f[2] : 0) + m3;
    for (int c = 0; c < 3; ++c) Q[c] = c1 * pb.B[c] + c2 * pb.B[3 + c] + c3 * pb.B[6 + c];
    q2 = Q[0] * Q[0] + Q[1] * Q[1] + Q[2] * Q[2];
    return true;
  }

  // Exchange-type tables at Q = Delta + G: V2a parallel (Q = 0: 1/r dropped, L(0) - W(0)), u~ (Q = 0: 0).
  // GRADIENT variant: V2a - L~ (Q != 0: 4 pi/Q^2 - W), ADJOINT: V2a - 2 L~; Q = 0 unchanged.
  static void fill_delta(const Problem& pb, const TableVariant& tv, const double* f, double scale, R* V, R* U1,
                         R* U2) {
    const double lf = tv.lap_factor();
    const double V0 = scale * chan_eval(tv, pb.A, pb.C, 0, [](auto A, auto C) {
                        return -kFourPi * A - 2.0 * kPi * A * A / C;
                      });
    for (long r = 0; r < NR; ++r) {
      double Q[3], q2;
      if (!grid_q(pb, r, f, Q, q2)) {
        V[r] = U1[r] = U2[r] = R(0);
        continue;
      }
      if (q2 < 1e-20) {
        V[r] = R(V0);
        U1[r] = U2[r] = R(0);
        continue;
      }
      const Jk k0 = chan_kernels(tv, pb.A, pb.C, 0, q2);
      const Jk k1 = chan_kernels(tv, pb.A, pb.C, 1, q2);
      V[r] = R(scale * (kFourPi / q2 + lf * k0.lap - k0.w));
      U1[r] = R(scale * k0.u);
      U2[r] = R(scale * k1.u);
    }
  }

  // Runs body(i) for i in [0, n) on the host's cores.
  template <class F>
  static void parallel_for(int n, F&& body) {
    const int nt = std::max(1, std::min<int>(n, int(std::thread::hardware_concurrency())));
    std::vector<std::thread> th;
    for (int t = 0; t < nt; ++t)
      th.emplace_back([&, t] {
        for (int i = t; i < n; i += nt) body(i);
      });
    for (auto& x : th) x.join();
  }

  void upload_tables(const Problem& pb, const TableVariant& tv) override {
    const int nD = (2 * pb.n1 - 1) * (2 * pb.n2 - 1) * (2 * pb.n3 - 1);
    const double scale = 1.0 / (pb.omega * double(NR));
    std::vector<R> V(size_t(nD) * NR), U1(size_t(nD) * NR), U2(size_t(nD) * NR);
    std::vector<double> df(size_t(nD) * 3);
    const int e2 = 2 * pb.n2 - 1, e3 = 2 * pb.n3 - 1;
    // after the mesh differences: band k-points, Delta = k_b - k_q (all b, q) then k_q - k_b
    const int nBand = 2 * pb.nkb * pb.nk;
    V.resize(size_t(nD + nBand) * NR);
    U1.resize(V.size());
    U2.resize(V.size());
    df.resize(size_t(nD + nBand) * 3);
    parallel_for(nD + nBand, [&](int di) {
      double f[3];
      if (di < nD) {
        const int d1 = di / (e2 * e3) - (pb.n1 - 1), d2 = (di / e3) % e2 - (pb.n2 - 1), d3 = di % e3 - (pb.n3 - 1);
        f[0] = double(d1) / pb.n1;
        f[1] = double(d2) / pb.n2;
        f[2] = double(d3) / pb.n3;
      } else {
        const int x = di - nD, sgn = x < pb.nkb * pb.nk ? 1 : -1, y = x % (pb.nkb * pb.nk);
        const int b = y / pb.nk, q = y % pb.nk;
        double fq[3];
        pb.kfrac(q, fq);
        for (int c = 0; c < 3; ++c) f[c] = sgn * (pb.bk[3 * b + c] - fq[c]);
      }
      for (int c = 0; c < 3; ++c) df[3 * size_t(di) + c] = f[c];
      fill_delta(pb, tv, f, scale, &V[size_t(di) * NR], &U1[size_t(di) * NR], &U2[size_t(di) * NR]);
    });
    tV.alloc(V.size());
    tU1.alloc(U1.size());
    tU2.alloc(U2.size());
    dfr.alloc(df.size());
    TC_HIP(hipMemcpy(tV.p, V.data(), V.size() * sizeof(R), hipMemcpyHostToDevice));
    TC_HIP(hipMemcpy(tU1.p, U1.data(), U1.size() * sizeof(R), hipMemcpyHostToDevice));
    TC_HIP(hipMemcpy(tU2.p, U2.data(), U2.size() * sizeof(R), hipMemcpyHostToDevice));
    TC_HIP(hipMemcpy(dfr.p, df.data(), df.size() * sizeof(double), hipMemcpyHostToDevice));
    // Hartree tables (Delta = 0, G = 0 dropped); both spin channels summed for the working precision
    const double lf = tv.lap_factor();
    std::vector<R> HV(NR), HU(NR), HVp(NR), HVa(NR), HUp(NR), HUa(NR);
    std::vector<double> hu0(NR), hu1(NR);
    for (long r = 0; r < NR; ++r) {
      double Q[3], q2;
      if (!grid_q(pb, r, nullptr, Q, q2) || q2 < 1e-20) {
        HV[r] = HU[r] = HVp[r] = HVa[r] = HUp[r] = HUa[r] = R(0);
        hu0[r] = hu1[r] = 0;
        continue;
      }
      const Jk k0 = chan_kernels(tv, pb.A, pb.C, 0, q2);
      const Jk k1 = chan_kernels(tv, pb.A, pb.C, 1, q2);
      const double v = kFourPi / q2;
      const double l0 = lf * k0.lap, l1 = lf * k1.lap;
      HV[r] = R(scale * ((v + l0 - k0.w) + (v + l1 - k1.w)));
      HU[r] = R(scale * (k0.u + k1.u));
      HVp[r] = R(scale * (v + l0 - k0.w));
      HVa[r] = R(scale * (v + l1 - k1.w));
      HUp[r] = R(scale * k0.u);
      HUa[r] = R(scale * k1.u);
      hu0[r] = scale * k0.u;
      hu1[r] = scale * k1.u;
    }
    tHV.alloc(NR);
    tHU.alloc(NR);
    tHu0.alloc(NR);
    tHu1.alloc(NR);
    TC_HIP(hipMemcpy(tHV.p, HV.data(), NR * sizeof(R), hipMemcpyHostToDevice));
    for (auto* b : {&tHVp, &tHVa, &tHUp, &tHUa}) b->alloc(NR);
    TC_HIP(hipMemcpy(tHVp.p, HVp.data(), NR * sizeof(R), hipMemcpyHostToDevice));
    TC_HIP(hipMemcpy(tHVa.p, HVa.data(), NR * sizeof(R), hipMemcpyHostToDevice));
    TC_HIP(hipMemcpy(tHUp.p, HUp.data(), NR * sizeof(R), hipMemcpyHostToDevice));
    TC_HIP(hipMemcpy(tHUa.p, HUa.data(), NR * sizeof(R), hipMemcpyHostToDevice));
    TC_HIP(hipMemcpy(tHU.p, HU.data(), NR * sizeof(R), hipMemcpyHostToDevice));
    TC_HIP(hipMemcpy(tHu0.p, hu0.data(), NR * sizeof(double), hipMemcpyHostToDevice));
    TC_HIP(hipMemcpy(tHu1.p, hu1.data(), NR * sizeof(double), hipMemcpyHostToDevice));
    // correction prefactors: A (Eqs. divcor_3a2_second, 3b6_div_scf2/3; the 2bx1 remainder of TC_DIV_LIMIT) and
    // A [4 pi A Delta_GB + nu u~_short(0)/N_k] with u~_short(0) = -4 pi A C^2 (Eqs. u_short, divcor_3a2_first,
    // 3b6_div_scf1): nu = 1 as printed; nu = 2 for TC_DIV_LIMIT, where the finite Q -> 0 remainder of
    // Q^2 u~(Q)^2 holds both cross terms of (4 pi A/Q^2 + u~_short)(4 pi A + Q^2 u~_short).
    const double nu = pb.reading == TC_DIV_LIMIT ? 2.0 : 1.0;
    for (int ch = 0; ch < 2; ++ch) {
      corrA[ch] = chan_eval(tv, pb.A, pb.C, ch, [](auto A, auto) { return A; });
      corrB[ch] = chan_eval(tv, pb.A, pb.C, ch, [&](auto A, auto C) {
        return A * (kFourPi * A * pb.delta_gb - nu * kFourPi * A * C * C / double(pb.nk));
      });
    }
  }

  // z stage: register FFTs, or split-BF16 MFMA DFTs (FP32 working precision, N divisible by 8)
  bool zmfma = false;
  DBuf<short> zfrag;   // [dir][hi/lo][mt][kt][lane][4] BF16 bits of the real 2N x 2N DFT matrices

  static uint16_t bf16_rne(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
  }
  static float bf16_val(uint16_t h) {
    const uint32_t u = uint32_t(h) << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
  }

  void upload_zfrag() {
    if constexpr (std::is_same<R, float>::value && N % 8 == 0) {
      constexpr int NT = ZMfma<N>::NT;
      std::vector<short> f(size_t(ZMfma<N>::NFRAG) * 4);
      for (int dir = 0; dir < 2; ++dir) {
        const double sgn = dir == 0 ? -1.0 : 1.0;   // forward e^{-2 pi i z'z/N}, inverse e^{+...}
        auto M = [&](int row, int col) {
          const int zp = row / 2, cp = row % 2, z = col / 2, c = col % 2;
          const double a = sgn * 2.0 * kPi * double((long(zp) * z) % N) / N;
          const double wr = std::cos(a), wi = std::sin(a);
          return cp == 0 ? (c == 0 ? wr : -wi) : (c == 0 ? wi : wr);
        };
        for (int mt = 0; mt < NT; ++mt)
          for (int kt = 0; kt < NT; ++kt)
            for (int l = 0; l < 64; ++l)
              for (int j = 0; j < 4; ++j) {
                const double v = M(16 * mt + l % 16, 16 * kt + 4 * (l / 16) + j);
                const uint16_t hi = bf16_rne(float(v));
                const uint16_t lo = bf16_rne(float(v - double(bf16_val(hi))));
                f[size_t(ZMfma<N>::frag(dir, 0, mt, kt) + l) * 4 + j] = short(hi);
                f[size_t(ZMfma<N>::frag(dir, 1, mt, kt) + l) * 4 + j] = short(lo);
              }
      }
      zfrag.alloc(f.size());
      TC_HIP(hipMemcpy(zfrag.p, f.data(), f.size() * sizeof(short), hipMemcpyHostToDevice));
    }
  }

  template <int OP>
  void zconv(hipStream_t s, const cx<R>* in, cx<R>* out, long npair, int t0, const MeshInfo& mi, const Tables& tb,
             int sign, const cx<R>* inB = nullptr) {
    if constexpr (std::is_same<R, float>::value && N % 8 == 0) {
      if (zmfma) {
        const long groups = npair * (long(N) * N / 16);
        const unsigned nb = unsigned(std::min<long>((groups + 3) / 4, 8192));
        hipLaunchKernelGGL((k_zconv_mfma<N, OP>), dim3(nb), dim3(256), 0, s, in, out, npair, t0, mi, tb, sign,
                           reinterpret_cast<const bf16x4*>(zfrag.p), inB);
        return;
      }
    }
    if constexpr (N == 48) {   // each column on a lane pair
      hipLaunchKernelGGL((k_zconv48<R, OP>), dim3(nblk(2 * npair * N * N)), dim3(256), 0, s, in, out, npair, t0, mi,
                         tb, sign, inB);
      return;
    }
    hipLaunchKernelGGL((k_zconv<R, N, OP>), dim3(nblk(npair * N * N)), dim3(256), 0, s, in, out, npair, t0, mi, tb,
                       sign, inB);
  }
  template <int OP>
  void zconv(hipStream_t s, long npair, int t0, const MeshInfo& mi, const Tables& tb, int sign) {
    zconv<OP>(s, bufA.p, bufB.p, npair, t0, mi, tb, sign);
  }

  void release_pair_store() override {
    allB.release();
    store_cap_ = INT_MAX;
  }

  // Bytes of per-batch pair buffers (bufA, bufB) of one target, and of the smallest batch worth keeping
  // next to the resident store
  static size_t per_target_bytes(const Problem& pb) {
    return size_t(pb.P()) * ((pb.bitc ? 8 : 5) + 4) * NR * sizeof(cx<R>);
  }
  // Bytes of bufA and bufB at a pair budget (the batch of ensure)
  static size_t batch_bytes(const Problem& pb, size_t budget_bytes) {
    const size_t per_t = per_target_bytes(pb), P = size_t(std::max(1, pb.P()));
    size_t T = std::max<size_t>(1, std::min(P, budget_bytes / per_t));
    if (pb.batch > 0) T = std::min(size_t(pb.batch), P);
    return T * per_t;
  }

  // The resident store of pass-A z-stage outputs, [pair][5] fields per spin channel, of the first Q1 partner
  // columns.  TC mode: triangular rows, the pairs (t, q) with q <= t and q < Q1 (tri_row; the pair (t, q) of
  // q > t is the reflected conjugate of (q, t)), so every pair with min(t, q) < Q1 is available; the
  // occupied pass reads it for its rows a < Q1 and forms its own pairs for the others, and pass A forms the
  // pairs of the targets and partners at or above Q1.  Biorthogonal mode: [t][P][5], every pair (the two
  // orders of a pair are not conjugate there) or none.  Q1 = P when every pair fits.  Without a caller budget it may take what leaves an eighth of the
  // device (at least 16 GiB) free once the batch buffers that follow it are allocated, the store it
  // already holds counted as free, and it keeps using every column it holds; with a budget
  // (tc_set_memory_budget), what leaves a batch of 8 targets of pair buffers.  Fewer than an eighth of the
  // columns are not worth the split passes: no store then.  Never under the no-allocation scratch.
  // Returns Q1 (0: no store).
  int pair_store(const Problem& pb) {
    const int P = pb.P();
    if (t_arena) return 0;
    auto none = [&] {
      allB.release();
      return 0;
    };
    if (!pb.pair_store || P == 0) return none();
    const int key = (P * 2 + int(pb.bitc)) * 2 + pb.nspin - 1;
    if (key != cap_key_) {   // the cap counts columns of one problem shape
      store_cap_ = INT_MAX;
      cap_key_ = key;
    }
    // elements of the store with Q1 partner columns: triangular rows in TC mode, P x Q1 in the biorthogonal one
    const size_t per_pair = size_t(5) * pb.nspin * NR;
    auto elems = [&](int q1) { return per_pair * (pb.bitc ? size_t(P) * q1 : size_t(tri_row(P, q1))); };
    auto fit = [&](size_t bytes) {   // most columns within bytes
      int q = 0;
      while (q < P && elems(q + 1) * sizeof(cx<R>) <= bytes) ++q;
      return q;
    };
    size_t avail = 0;
    if (pb.mem_budget) {
      const size_t keep = per_target_bytes(pb) * std::min(8, P);
      avail = pb.mem_budget > keep ? pb.mem_budget - keep : 0;
    } else {
      size_t fr = 0, tot = 0;
      if (hipMemGetInfo(&fr, &tot) != hipSuccess) return none();
      const size_t have = allB.p ? allB.n * sizeof(cx<R>) : 0;
      // the batch buffers are sized after the store: what they still have to take counts as taken
      const size_t held = ((bufA.p ? bufA.n : 0) + (bufB.p ? bufB.n : 0)) * sizeof(cx<R>);
      const size_t want = batch_bytes(pb, pair_budget(pb));
      const size_t reserve = std::max<size_t>(tot / 8, size_t(16) << 30) + (want > held ? want - held : 0);
      avail = fr + have > reserve ? fr + have - reserve : 0;
    }
    int q1 = fit(avail);
    if (!pb.mem_budget && allB.p) q1 = std::max(q1, fit(allB.n * sizeof(cx<R>)));
    q1 = std::min(q1, store_cap_);   // a size that failed is not asked for again
    if (pb.bitc && q1 < P) q1 = 0;
    if (q1 < (P + 7) / 8) return none();
    if (allB.n >= elems(q1)) return q1;
    allB.release();
    // on failure: fewer columns, down to the fewest worth keeping
    for (; q1 >= (P + 7) / 8 && (!pb.bitc || q1 == P); q1 -= std::max(1, P / 16)) {
      try {
        allB.alloc(elems(q1));
        return q1;
      } catch (const TcError&) {
        store_cap_ = q1 - 1;
      }
    }
    return 0;
  }
  int store_cap_ = INT_MAX;   // most partner columns an allocation may still ask for (at the shape cap_key_)
  int cap_key_ = -1;

  // Bytes of per-batch pair buffers.  Without a caller budget: an eighth of the device's memory, between
  // 8 and 32 GiB (32 GiB on a 288 GB device: 134 targets per batch at 256 orbitals and 24^3 in FP32);
  // larger batches mean fewer, larger launches and fewer partial tails.  With a budget: what the store
  // leaves of it, at most 32 GiB.  Under the no-allocation scratch: a third of what is left of it.
  size_t budget_ = 0;
  size_t pair_budget(const Problem& pb) {
    if (t_arena) return (t_arena->cap - t_arena->used) / 3;
    if (pb.mem_budget) {
      const size_t store = allB.p ? allB.n * sizeof(cx<R>) : 0;
      return std::min(size_t(32) << 30, pb.mem_budget > store ? pb.mem_budget - store : size_t(0));
    }
    if (!budget_) {
      size_t fr = 0, tot = 0;
      if (hipMemGetInfo(&fr, &tot) != hipSuccess) tot = 0;
      budget_ = std::min(size_t(32) << 30, std::max(size_t(8) << 30, tot / 8));
    }
    return budget_;
  }

  size_t budget_alloc = size_t(-1);
  void ensure(const Problem& pb, size_t budget_bytes) {
    const int P = pb.P();
    // under the no-allocation scratch every buffer is bound to it again
    if (!t_arena && P == P_alloc && pb.batch == batch_alloc && pb.bitc == bitc_alloc && pb.nspin == nspin_alloc &&
        budget_bytes == budget_alloc)
      return;
    if (t_arena) t_arena->undo.push_back([this, T0 = T, S0 = S] {   // the batch shape of the ordinary buffers
      T = T0;
      S = S0;
    });
    psi.alloc(size_t(P) * NR);
    D.alloc(size_t(3) * P * NR);
    Dl.alloc(size_t(3) * P * NR);
    Hl.alloc(size_t(3) * P * NR);
    nJ.alloc(4 * NR);
    loc.alloc(8 * NR);
    wk.alloc(9 * NR);
    H3a4.alloc(size_t(3) * P * NR);
    h5.alloc(size_t(P) * NR);
    // per target: 4 pair fields in bufA and 5 in bufB (8 in biorthogonal mode: V21 and V12 of the
    // occupied-occupied pass)
    const int nB = pb.bitc ? 8 : 5;
    const size_t per_t = per_target_bytes(pb);
    T = int(std::max<size_t>(1, std::min<size_t>(size_t(P), budget_bytes / per_t)));
    if (pb.batch > 0) T = std::min(pb.batch, P);
    for (;;) {
      try {
        bufA.alloc(size_t(T) * P * 4 * NR);
        bufB.alloc(size_t(T) * P * nB * NR);
        break;
      } catch (const TcError& e) {
        // the device is fuller than its free memory said (another context, the caller's tensors): fewer
        // targets per batch, which changes no result
        if (t_arena || T == 1 || e.code != TC_ERR_OOM) throw;
        bufA.release();
        bufB.release();
        T = (T + 1) / 2;
      }
    }
    h4.alloc(size_t(3) * T * NR);
    Z.alloc(size_t(3) * T * NR);
    g.alloc(size_t(T) * NR);
    acc.alloc(size_t(kAccSlots) * T * NR);
    // partner chunks: enough work-groups (targets x z-planes x chunks) to fill the chip,
    // at most 64 partners per chunk (working-precision partial sums)
    S = int(std::min<long>(P, std::max<long>({1L, (2048 + long(T) * N - 1) / (long(T) * N), (P + 63L) / 64})));
    gpart.alloc(size_t(S) * 3 * T * NR);
    h4part.alloc(size_t(S) * 3 * T * NR);
    h5part.alloc(size_t(S) * T * NR);
    H3part.alloc(size_t(S) * 3 * T * NR);
    psi64.alloc(size_t(P) * NR);
    v64.alloc(4 * NR);
    prod64.alloc(size_t(2) * P * NR);
    focc.alloc(P);
    if (pb.bitc) {
      chi.alloc(size_t(P) * NR);
      H3bc.alloc(size_t(3) * P * NR);
      h5c.alloc(size_t(P) * NR);
      h5cpart.alloc(size_t(S) * T * NR);
      Hbpart.alloc(size_t(S) * 3 * T * NR);
      chi64.alloc(size_t(P) * NR);
    }
    if (pb.nspin == 2) {
      psi1.alloc(size_t(P) * NR);
      D1.alloc(size_t(3) * P * NR);
      Dl1.alloc(size_t(3) * P * NR);
      Hl1.alloc(size_t(3) * P * NR);
      H3a4_1.alloc(size_t(3) * P * NR);
      nJ1.alloc(4 * NR);
      loc1.alloc(8 * NR);
      wk2.alloc(16 * NR);
      h5_1.alloc(size_t(P) * NR);
      h5a0.alloc(size_t(P) * NR);
      h5a1.alloc(size_t(P) * NR);
      h5part.alloc(size_t(2) * S * T * NR);
      psi64_1.alloc(size_t(P) * NR);
      v64p.alloc(10 * NR);
      if (pb.bitc) {
        chi1.alloc(size_t(P) * NR);
        H3bc_1.alloc(size_t(3) * P * NR);
        h5c_1.alloc(size_t(P) * NR);
        h5ca0.alloc(size_t(P) * NR);
        h5ca1.alloc(size_t(P) * NR);
        h5cpart.alloc(size_t(2) * S * T * NR);
        chi64_1.alloc(size_t(P) * NR);
      }
    }
    if (t_arena) return;   // the buffers of the no-allocation call are unbound when it ends
    P_alloc = P;
    batch_alloc = pb.batch;
    bitc_alloc = pb.bitc;
    nspin_alloc = pb.nspin;
    budget_alloc = budget_bytes;
  }

  // One application of the operator (Sec. 2.6, the six stages above) for one or two spin channels
  // (Sec. 2.1, Eq. SCF: one orbital set per spin), in TC mode or the biorthogonal mode (the left orbitals
  // chi as bras), with the orbitals, trial vectors (ts) or band orbitals (ts->band) as targets.  With two
  // channels the Hartree-type fields of target spin s take the parallel tables on its own density and the
  // antiparallel ones on the other's, exchange-type terms pair orbitals of one spin, and the occupied pass
  // keeps the parallel and antiparallel parts of h5 apart: h6 of spin s sums the first over own-spin rows
  // and the second over other-spin rows.  With crystal symmetry (TC mode, one channel) the rows of the
  // occupied-occupied pass (q2 of Algs. 3a2, 3a4, 3b2) and the targets are the orbitals of the
  // representative k-points only: h5 and H3a4 of the other orbitals follow from the representatives' by the
  // grid permutation of their operation (k_sym_fields), their outputs and energy slots likewise (k_sym_coef,
  // k_sym_epart); densities, partner sums and corrections use every orbital.
  void apply(hipStream_t s, Shared& sh, const Problem& pb, double* stage_ms, const TargetSet* ts) override {
    const int P = pb.P();
    const int nb = pb.nb;
    const int ns = pb.nspin;
    const bool pol = ns == 2;
    const bool sym = pb.nsym > 0;   // TC mode, one channel, orbitals as targets (checked at preparation)
    const int PI = sym ? int(pb.irr.size()) * nb : P;   // the representatives' orbitals
    Masks m = make_masks(pb.mask);
    if (pb.negate_b) {   // v2 -> v2^dagger: the grad-u . grad terms change sign (with the ADJOINT tables)
      m.m2bh1 = -m.m2bh1;
      m.m2bh2 = -m.m2bh2;
      m.m2bx1 = -m.m2bx1;
      m.m2bx2 = -m.m2bx2;
    }
    const bool need_occ = m.m3a2 || m.m3a4 || m.m3b2 || m.m3b5;
    const bool need_A = m.m2ax || m.m2bx1 || m.m2bx2 || m.m3a3 || m.m3a4 || m.m3b4 || m.m3b6;
    const bool need_B = m.m2bx2 || m.m3b3 || m.m3b4 || m.m3b5;
    // With the orbitals as targets, the pass-A pair (t = b, q = a) has the density conj(psi_a) psi_b and the
    // momentum Delta = k_b - k_a of the occupied pair (a, b), and the four fields of its z stage after V are
    // the occupied pass's.  When every pair's pass-A z-stage output fits on the device (one region per spin
    // channel) it is computed once, before the occupied pass, which then reads it in place of its own pair
    // densities and z stage.  (The store is settled before the batch buffers, which take what it leaves of a
    // caller's budget.)
    const int Q1 = (!ts && !sym && need_occ && need_A) ? pair_store(pb) : 0;   // stored partner columns
    const bool keepA = Q1 > 0;
    const bool tri = keepA && !pb.bitc;   // TC mode: the triangular store (tri_row)
    // TC mode with the store (one or two channels): h5 of Alg. 3a2 comes from pass A (k_fused_A<H5A>), whose targets are
    // the occupied pass's rows and whose pair fields are the conjugates of the occupied pass's, so the occupied
    // pass transforms the parallel channel only (H3a4).  h6 is then complete after the last target batch, and
    // its local term is applied to every target after the batches (k_h6_sum, k_h6_apply, k_h6_energy).
    const bool h5A = tri && m.m3a2 != 0;
    ensure(pb, pair_budget(pb));
    // targets: the orbitals, or nbt trial vectors per k-point
    const int nbt = ts ? ts->nvec : nb;
    const int NTG = sym ? PI : (ts && ts->nblk ? ts->nblk : pb.nk) * nbt;
    // occupied-occupied pass and target passes (with symmetry: rows and targets are the representatives)
    const MeshInfo mi = sym ? MeshInfo{pb.n1, pb.n2, pb.n3, nb, P, nb, sh.irrk.p} : MeshInfo{pb.n1, pb.n2, pb.n3, nb, P, nb};
    const MeshInfo miT = sym ? mi : MeshInfo{pb.n1, pb.n2, pb.n3, nb, P, nbt, ts ? ts->tk : nullptr, pb.nkb};
    // plane-wave data of the targets (band targets carry their own)
    const bool tb_own = ts && ts->boxidx;
    const int* tbox = tb_own ? ts->boxidx : sh.boxidx.p;
    const int* tnpw = tb_own ? ts->npw : sh.npw.p;
    const double* tkg = tb_own ? ts->kg : sh.kg.p;
    const int tnpm = tb_own ? ts->npm : pb.npw_max;
    Recip rc;
    for (int i = 0; i < 9; ++i) rc.b[i] = pb.B[i];
    Basis<R> bm, mm;   // B_dc = (b_d)_c and the metric M = B B^T, working precision
    for (int i = 0; i < 9; ++i) bm.b[i] = R(pb.B[i]);
    for (int d = 0; d < 3; ++d)
      for (int e = 0; e < 3; ++e)
        mm.b[3 * d + e] = R(pb.B[3 * d] * pb.B[3 * e] + pb.B[3 * d + 1] * pb.B[3 * e + 1] + pb.B[3 * d + 2] * pb.B[3 * e + 2]);
    const Tables tb{tV.p, tU1.p, tU2.p, dfr.p};
    const bool bitc = pb.bitc;
    // per-channel fields (the second of each pair only with two channels); bras: the left orbitals chi in
    // the biorthogonal mode, psi in TC mode
    cx<R>* PSI[2] = {psi.p, psi1.p};
    cx<R>* DD[2] = {D.p, D1.p};
    cx<R>* DL[2] = {Dl.p, Dl1.p};
    cx<R>* HL[2] = {Hl.p, Hl1.p};
    cx<R>* H3[2] = {H3a4.p, H3a4_1.p};
    cx<R>* NJ[2] = {nJ.p, nJ1.p};
    cx<R>* LOC[2] = {loc.p, loc1.p};
    cx<R>* CHI[2] = {chi.p, chi1.p};
    const cx<R>* XS[2] = {bitc ? chi.p : psi.p, bitc ? chi1.p : psi1.p};
    R* H5P[2] = {h5.p, h5_1.p};          // real h5 (TC); with two channels its parallel-channel part
    R* H5A[2] = {h5a0.p, h5a1.p};        // antiparallel-channel part (two channels)
    cx<R>* H5C[2] = {h5c.p, h5c_1.p};    // the same, complex (biorthogonal mode)
    cx<R>* H5CA[2] = {h5ca0.p, h5ca1.p};
    cx<R>* HBC[2] = {H3bc.p, H3bc_1.p};  // conj(H3b), then its lattice components (biorthogonal mode)
    const double* W[2] = {sh.w.p, sh.w.p + P};
    const size_t cofs = size_t(2) * P * pb.npw_max;   // doubles per channel of the coefficients
    const size_t tcofs = size_t(2) * NTG * tnpm;      // doubles per channel of the target coefficients
    // the resident store of channel c: pass-A z-stage outputs [pair][5][N^3], pair-major in target order;
    // triangular rows in TC mode, [P][Q1] in the biorthogonal mode
    const size_t spairs = tri ? size_t(tri_row(P, Q1)) : size_t(P) * Q1;
    auto store = [&](int c) { return allB.p + size_t(c) * spairs * 5 * NR; };
    // algorithmic bytes: fields each launch must read or write once (working precision)
    const double fb = double(sizeof(cx<R>)) * NR;
    const double fd = double(sizeof(cx<double>)) * NR;
    const double tabB = 3.0 * double(sizeof(R)) * NR * double((2 * pb.n1 - 1) * (2 * pb.n2 - 1) * (2 * pb.n3 - 1));
    Prof* pf = prof;
    auto K = [&](int id, double bytes, auto&& launch) {
      ProfScope ps(pf, s, id, bytes);
      launch();
    };
    Events ev(6);
    std::vector<hipEvent_t> bev;   // per batch: begin A, end A, end B
    ev.rec(0, s);

    // ---- 0: G -> r (psi, the three components of D, and chi in the biorthogonal mode), per channel
    const unsigned gsc = nblk(long(P) * pb.npw_max);
    for (int c = 0; c < ns; ++c) {
      const double* cf = sh.coef.p + c * cofs;
      TC_HIP(hipMemsetAsync(PSI[c], 0, size_t(P) * NR * sizeof(cx<R>), s));
      TC_HIP(hipMemsetAsync(DD[c], 0, size_t(3) * P * NR * sizeof(cx<R>), s));
      if (bitc) TC_HIP(hipMemsetAsync(CHI[c], 0, size_t(P) * NR * sizeof(cx<R>), s));
      K(TC_K_SCATTER, 0.0, [&] {
        hipLaunchKernelGGL((k_scatter<R>), dim3(gsc), dim3(256), 0, s, cf, sh.boxidx.p, sh.npw.p, sh.kg.p, nb,
                           pb.npw_max, P, -1, PSI[c], NR);
        for (int d = 0; d < 3; ++d)
          hipLaunchKernelGGL((k_scatter<R>), dim3(gsc), dim3(256), 0, s, cf, sh.boxidx.p, sh.npw.p, sh.kg.p, nb,
                             pb.npw_max, P, d, DD[c] + size_t(d) * P * NR, NR);
        if (bitc)
          hipLaunchKernelGGL((k_scatter<R>), dim3(gsc), dim3(256), 0, s, sh.coefL.p + c * cofs, sh.boxidx.p,
                             sh.npw.p, sh.kg.p, nb, pb.npw_max, P, -1, CHI[c], NR);
      });
      fft3d_t<R, N>(PSI[c], P, +1, s, pf);
      if (bitc) fft3d_t<R, N>(CHI[c], P, +1, s, pf);
      fft3d_t<R, N>(DD[c], 3L * P, +1, s, pf);
      K(TC_K_OTHER, 6.0 * fb * P, [&] {
        hipLaunchKernelGGL((k_lattice3<R, N>), dim3(nblk(long(P) * NR)), dim3(256), 0, s, DD[c], DL[c], bm, long(P),
                           NR, long(P) * NR);
      });
    }
    // target fields of trial vectors or band orbitals (channel c's; with one channel made here, with two at
    // that channel's target passes)
    if (ts || sym) {
      psiT.alloc(size_t(NTG) * NR);
      DT.alloc(size_t(3) * NTG * NR);
    }
    if (sym) {   // the representatives' fields as rows and targets; their fields and outputs before expansion
      for (int i = 0; i < int(pb.irr.size()); ++i) {
        const size_t blk = size_t(nb) * NR, src = size_t(pb.irr[i]) * blk, dst = size_t(i) * blk;
        TC_HIP(hipMemcpyAsync(psiT.p + dst, psi.p + src, blk * sizeof(cx<R>), hipMemcpyDeviceToDevice, s));
        for (int d = 0; d < 3; ++d)
          TC_HIP(hipMemcpyAsync(DT.p + size_t(d) * PI * NR + dst, D.p + size_t(d) * P * NR + src, blk * sizeof(cx<R>),
                                hipMemcpyDeviceToDevice, s));
      }
      H3I.alloc(size_t(3) * PI * NR);
      h5I.alloc(size_t(PI) * NR);
      sh.outI.alloc(size_t(2) * PI * pb.npw_max);
      sh.epartI.alloc(size_t(kAccSlots) * PI);
    }
    auto scatter_targets = [&](int c) {
      TC_HIP(hipMemsetAsync(psiT.p, 0, size_t(NTG) * NR * sizeof(cx<R>), s));
      TC_HIP(hipMemsetAsync(DT.p, 0, size_t(3) * NTG * NR * sizeof(cx<R>), s));
      const unsigned gst = nblk(long(NTG) * tnpm);
      const double* tc = ts->coef + c * tcofs;
      K(TC_K_SCATTER, 0.0, [&] {
        hipLaunchKernelGGL((k_scatter<R>), dim3(gst), dim3(256), 0, s, tc, tbox, tnpw, tkg, nbt, tnpm, NTG, -1,
                           psiT.p, NR);
        for (int d = 0; d < 3; ++d)
          hipLaunchKernelGGL((k_scatter<R>), dim3(gst), dim3(256), 0, s, tc, tbox, tnpw, tkg, nbt, tnpm, NTG, d,
                             DT.p + size_t(d) * NTG * NR, NR);
      });
      fft3d_t<R, N>(psiT.p, NTG, +1, s, pf);
      fft3d_t<R, N>(DT.p, 3L * NTG, +1, s, pf);
    };
    if (ts && !pol) scatter_targets(0);
    ev.rec(1, s);

    // ---- 1: densities and Hartree-type fields (Algs. 2ah, 3a1, 3b1; 2bh1, 2bh2)
    if (!pol) {
      TC_HIP(hipMemsetAsync(loc.p, 0, 8 * NR * sizeof(cx<R>), s));
      K(TC_K_OTHER, fb * (4.0 * P + 4.0), [&] {
        hipLaunchKernelGGL((k_density<R, N>), dim3(nblk(NR)), dim3(256), 0, s, XS[0], psi.p, D.p, sh.w.p, P, nJ.p,
                           nJ.p + NR);
      });
      TC_HIP(hipMemcpyAsync(wk.p, nJ.p, 4 * NR * sizeof(cx<R>), hipMemcpyDeviceToDevice, s));
      fft3d_t<R, N>(wk.p, 4, -1, s, pf);
      K(TC_K_OTHER, fb * 9.0, [&] {
        hipLaunchKernelGGL((k_hartree_g<R, N>), dim3(nblk(NR)), dim3(256), 0, s, rc, tHV.p, tHU.p, wk.p, wk.p + NR,
                           wk.p + 4 * NR);
      });
      fft3d_t<R, N>(wk.p + 4 * NR, 5, +1, s, pf);
      TC_HIP(hipMemcpyAsync(loc.p, wk.p + 4 * NR, 5 * NR * sizeof(cx<R>), hipMemcpyDeviceToDevice, s));
      K(TC_K_OTHER, fb * 7.0, [&] {
        hipLaunchKernelGGL((k_mul_vec_scalar<R, N>), dim3(nblk(NR)), dim3(256), 0, s, loc.p + NR, nJ.p, wk.p);
      });
      fft3d_t<R, N>(wk.p, 3, -1, s, pf);
      K(TC_K_OTHER, fb * 4.0, [&] {
        hipLaunchKernelGGL((k_gdiv<R, N>), dim3(nblk(NR)), dim3(256), 0, s, rc, tHU.p, wk.p, wk.p + 3 * NR);
      });
      fft3d_t<R, N>(wk.p + 3 * NR, 1, +1, s, pf);
      TC_HIP(hipMemcpyAsync(loc.p + 5 * NR, wk.p + 3 * NR, NR * sizeof(cx<R>), hipMemcpyDeviceToDevice, s));
    } else {
      // wk2: [0..3] n~, J~ of channel 0, [4..7] of channel 1, [8..10] / [11..13] products or M per channel
      for (int sp = 0; sp < 2; ++sp) {
        TC_HIP(hipMemsetAsync(LOC[sp], 0, 8 * NR * sizeof(cx<R>), s));
        K(TC_K_OTHER, fb * (4.0 * P + 4.0), [&] {
          hipLaunchKernelGGL((k_density<R, N>), dim3(nblk(NR)), dim3(256), 0, s, XS[sp], PSI[sp], DD[sp], W[sp], P,
                             NJ[sp], NJ[sp] + NR);
        });
        TC_HIP(hipMemcpyAsync(wk2.p + 4 * sp * NR, NJ[sp], 4 * NR * sizeof(cx<R>), hipMemcpyDeviceToDevice, s));
      }
      fft3d_t<R, N>(wk2.p, 8, -1, s, pf);
      for (int sp = 0; sp < 2; ++sp) {
        const int o = 1 - sp;
        K(TC_K_OTHER, fb * 13.0, [&] {
          hipLaunchKernelGGL((k_hartree_g2<R, N>), dim3(nblk(NR)), dim3(256), 0, s, rc, tHVp.p, tHVa.p, tHUp.p, tHUa.p,
                             wk2.p + 4 * sp * NR, wk2.p + (4 * sp + 1) * NR, wk2.p + 4 * o * NR,
                             wk2.p + (4 * o + 1) * NR, wk.p);
        });
        fft3d_t<R, N>(wk.p, 5, +1, s, pf);
        TC_HIP(hipMemcpyAsync(LOC[sp], wk.p, 5 * NR * sizeof(cx<R>), hipMemcpyDeviceToDevice, s));
      }
      // 3b1: sum_s1 -i G . u^{s s1} FT(h1^{s1} n_{s1})
      for (int sp = 0; sp < 2; ++sp)
        K(TC_K_OTHER, fb * 7.0, [&] {
          hipLaunchKernelGGL((k_mul_vec_scalar<R, N>), dim3(nblk(NR)), dim3(256), 0, s, LOC[sp] + NR, NJ[sp],
                             wk2.p + (8 + 3 * sp) * NR);
        });
      fft3d_t<R, N>(wk2.p + 8 * NR, 6, -1, s, pf);
      for (int sp = 0; sp < 2; ++sp) {
        const int o = 1 - sp;
        K(TC_K_OTHER, fb * 7.0, [&] {
          hipLaunchKernelGGL((k_gdiv2<R, N>), dim3(nblk(NR)), dim3(256), 0, s, rc, tHUp.p, tHUa.p,
                             wk2.p + (8 + 3 * sp) * NR, wk2.p + (8 + 3 * o) * NR, wk.p);
        });
        fft3d_t<R, N>(wk.p, 1, +1, s, pf);
        TC_HIP(hipMemcpyAsync(LOC[sp] + 5 * NR, wk.p, NR * sizeof(cx<R>), hipMemcpyDeviceToDevice, s));
      }
    }
    ev.rec(2, s);

    // ---- 2: occupied-occupied pair pass (Algs. 3a2, 3a4 and 3b2/3b5 first loops), per channel
    const int chunk = (P + S - 1) / S;
    if (tri) {   // the pairs (t, q <= t, q < Q1) of every target, before the occupied pass
      for (int c = 0; c < ns; ++c)
        for (int t0 = 0; t0 < P; t0 += T) {
          const int nt = std::min(T, P - t0);
          const int qn = std::min(t0 + nt, Q1);   // partners formed for the batch: bufA [t][qn]
          const FusedArgs fa{qn, nt, t0, S, (qn + S - 1) / S};
          K(TC_K_XY_PAIR_TGT, fb * (double(nt) * qn + nt + qn), [&] {
            hipLaunchKernelGGL((k_pair_xy<R, N, false>), dim3(unsigned(nt) * N * S), dim3(NTH), 0, s, XS[c], PSI[c],
                               fa, bufA.p);
          });
          const long rows = tri_row(t0 + nt, Q1) - tri_row(t0, Q1);   // pairs the batch's rows hold
          K(TC_K_ZCONV_A1, fb * 6.0 * rows + tabB, [&] {   // row t0 + t: partners 0 .. min(t0 + t, Q1 - 1)
            MeshInfo miQ{pb.n1, pb.n2, pb.n3, nb, qn, nb};
            miQ.trq = Q1;
            zconv<OP_A1>(s, bufA.p, store(c) + size_t(tri_row(t0, Q1)) * 5 * NR, rows, t0, miQ, tb, 1);
          });
        }
    } else if (keepA) {   // the pairs (t, q < Q1) of every target, before the occupied pass
      const MeshInfo miQ{pb.n1, pb.n2, pb.n3, nb, Q1, nb};
      const int chunkQ = (Q1 + S - 1) / S;
      for (int c = 0; c < ns; ++c)
        for (int t0 = 0; t0 < P; t0 += T) {
          const int nt = std::min(T, P - t0);
          const long npair = long(nt) * Q1;
          const FusedArgs fa{Q1, nt, t0, S, chunkQ};
          K(TC_K_XY_PAIR_TGT, fb * (npair + nt + Q1), [&] {
            hipLaunchKernelGGL((k_pair_xy<R, N, false>), dim3(unsigned(nt) * N * S), dim3(NTH), 0, s, XS[c], PSI[c],
                               fa, bufA.p);
          });
          K(TC_K_ZCONV_A1, fb * 6.0 * npair + tabB, [&] {
            zconv<OP_A1>(s, bufA.p, store(c) + size_t(t0) * Q1 * 5 * NR, npair, t0, miQ, tb, 1);
          });
        }
    }
    for (int c = 0; c < ns; ++c) {
      TC_HIP(hipMemsetAsync(H3[c], 0, size_t(3) * P * NR * sizeof(cx<R>), s));
      if (bitc) TC_HIP(hipMemsetAsync(HBC[c], 0, size_t(3) * P * NR * sizeof(cx<R>), s));
      if (sym) TC_HIP(hipMemsetAsync(h5.p, 0, size_t(P) * NR * sizeof(R), s));
      if (pol && bitc) {
        TC_HIP(hipMemsetAsync(H5C[c], 0, size_t(P) * NR * sizeof(cx<R>), s));
        TC_HIP(hipMemsetAsync(H5CA[c], 0, size_t(P) * NR * sizeof(cx<R>), s));
      } else if (pol) {
        TC_HIP(hipMemsetAsync(H5P[c], 0, size_t(P) * NR * sizeof(R), s));
        TC_HIP(hipMemsetAsync(H5A[c], 0, size_t(P) * NR * sizeof(R), s));
      }
    }
    if (need_occ) {
      for (int c = 0; c < ns; ++c)
        for (int a0 = 0, nt = 0; a0 < PI; a0 += nt) {
          // rows below Q1 read the store (a batch never straddles Q1); the others form their own pairs
          const bool stored = keepA && a0 < Q1;
          nt = std::min(T, (stored ? Q1 : PI) - a0);
          const long npair = long(nt) * P;
          const FusedArgs fa{P, nt, a0, S, chunk};
          if (bitc) {
            // row a = a0 + t, partner b = q: V21 from rho21 = conj(chi_a) psi_b at Delta = k_b - k_a, V12 from
            // rho12 = conj(chi_b) psi_a at Delta = k_a - k_b (no conjugate symmetry between them); with the
            // store they are its pairs b P + a and a P + b, fields 1..4
            const cx<R>* b21 = bufB.p;
            const cx<R>* b12 = bufB.p + 4 * npair * NR;
            long sT21 = -1, sQ21 = 4, sT12 = -1, sQ12 = 4;
            if (stored) {   // Q1 = P in the biorthogonal mode
              b21 = store(c) + (size_t(a0) * 5 + 1) * NR;
              b12 = store(c) + (size_t(a0) * 5 * Q1 + 1) * NR;
              sT21 = 5;
              sQ21 = 5L * Q1;
              sT12 = 5L * Q1;
              sQ12 = 5;
            } else {
              cx<R>* in12 = bufA.p + npair * NR;
              cx<R>* out12 = bufB.p + 4 * npair * NR;
              K(TC_K_XY_PAIR_OCC, fb * 2.0 * (npair + nt + P), [&] {
                hipLaunchKernelGGL((k_pair_xy<R, N, true>), dim3(unsigned(nt) * N * S), dim3(NTH), 0, s, XS[c],
                                   PSI[c], fa, bufA.p);
                hipLaunchKernelGGL((k_pair_xy<R, N, false>), dim3(unsigned(nt) * N * S), dim3(NTH), 0, s, XS[c],
                                   PSI[c], fa, in12);
              });
              K(TC_K_ZCONV_OCC, 2.0 * (fb * 5.0 * npair + tabB), [&] {
                zconv<OP_O>(s, bufA.p, bufB.p, npair, a0, mi, tb, 0);
                zconv<OP_O>(s, in12, out12, npair, a0, mi, tb, 1);
              });
            }
            K(TC_K_FUSED_OB, fb * (8.0 * npair + 2.0 * P) + (pol ? 8.0 : 7.0) * fb * nt * S, [&] {
              if (pol)
                hipLaunchKernelGGL((k_fused_OB<R, N, true>), dim3(unsigned(nt) * N * S), dim3(NTH), 0, s, b21, b12,
                                   PSI[c], XS[c], W[c], fa, mi, rc, dfr.p, h5cpart.p, H3part.p, Hbpart.p, sT21, sQ21,
                                   sT12, sQ12);
              else
                hipLaunchKernelGGL((k_fused_OB<R, N>), dim3(unsigned(nt) * N * S), dim3(NTH), 0, s, b21, b12, PSI[c],
                                   XS[c], W[c], fa, mi, rc, dfr.p, h5cpart.p, H3part.p, Hbpart.p, sT21, sQ21, sT12,
                                   sQ12);
            });
            K(TC_K_SUM_PARTS, (pol ? 8.0 : 7.0) * fb * nt * (S + 1), [&] {
              hipLaunchKernelGGL((k_sum_parts_ob<R, N>), dim3(nblk(long(nt) * NR)), dim3(256), 0, s, S, nt, a0,
                                 h5cpart.p, H3part.p, Hbpart.p, H5C[c], H3[c], HBC[c]);
              if (pol)   // the antiparallel-channel part (second half of the partials)
                hipLaunchKernelGGL((k_sum_cx_parts<R, N>), dim3(nblk(long(nt) * NR)), dim3(256), 0, s, S, nt, a0,
                                   h5cpart.p + size_t(S) * nt * NR, H5CA[c]);
            });
          } else {
            // row a = a0 + t, partner b = q; from the store: fields 1..4 of its pair (b, a), or of (a, b)
            // reflected and conjugated (triangular store)
            const cx<R>* b4 = bufB.p;
            const cx<R>* trs = stored ? store(c) : nullptr;
            long sT = -1, sQ = 4;
            if (!stored) {
              K(TC_K_XY_PAIR_OCC, fb * (npair + nt + P), [&] {
                hipLaunchKernelGGL((k_pair_xy<R, N, true>), dim3(unsigned(nt) * N * S), dim3(NTH), 0, s,
                                   sym ? psiT.p : PSI[c], PSI[c], fa, bufA.p);
              });
              K(TC_K_ZCONV_OCC, fb * 5.0 * npair + tabB, [&] {
                zconv<OP_O>(s, npair, a0, mi, tb, 0);
              });
            }
            K(TC_K_FUSED_O, fb * ((h5A ? 2.0 : 4.0) * npair + P) + (pol ? 4.5 : 3.5) * fb * nt * S, [&] {
              if (pol && h5A)
                hipLaunchKernelGGL((k_fused_O<R, N, true, false>), dim3(unsigned(nt) * N * S), dim3(NTH), 0, s, b4,
                                   PSI[c], W[c], fa, mi, rc, dfr.p, h5part.p, H3part.p, sT, sQ, trs, Q1);
              else if (pol)
                hipLaunchKernelGGL((k_fused_O<R, N, true>), dim3(unsigned(nt) * N * S), dim3(NTH), 0, s, b4, PSI[c],
                                   W[c], fa, mi, rc, dfr.p, h5part.p, H3part.p, sT, sQ, trs, Q1);
              else if (h5A)
                hipLaunchKernelGGL((k_fused_O<R, N, false, false>), dim3(unsigned(nt) * N * S), dim3(NTH), 0, s, b4,
                                   PSI[c], W[c], fa, mi, rc, dfr.p, h5part.p, H3part.p, sT, sQ, trs, Q1);
              else
                hipLaunchKernelGGL((k_fused_O<R, N>), dim3(unsigned(nt) * N * S), dim3(NTH), 0, s, b4, PSI[c], W[c],
                                   fa, mi, rc, dfr.p, h5part.p, H3part.p, sT, sQ, trs, Q1);
            });
            K(TC_K_SUM_PARTS, (pol ? 5.0 : 4.0) * fb * nt * (S + 1), [&] {
              hipLaunchKernelGGL((k_sum_parts<R, N>), dim3(nblk(long(nt) * NR)), dim3(256), 0, s, 0, S, nt, a0, 0,
                                 h5part.p, H3part.p, nullptr, nullptr, sym ? h5I.p : H5P[c], sym ? H3I.p : H3[c],
                                 nullptr, nullptr);
              if (pol)   // the antiparallel-channel part (second half of the partials)
                hipLaunchKernelGGL((k_sum_real_parts<R, N>), dim3(nblk(long(nt) * NR)), dim3(256), 0, s, S, nt, a0,
                                   h5part.p + size_t(S) * nt * NR, H5A[c]);
            });
          }
        }
      if (sym)   // every orbital's h5 and H3a4 from its representative's
        K(TC_K_OTHER, fb * 4.0 * (P + PI), [&] {
          hipLaunchKernelGGL((k_sym_fields<R, N>), dim3(nblk(long(P) * NR)), dim3(256), 0, s, sh.symk.p, nb, P, h5I.p,
                             H3I.p, h5.p, H3a4.p);
        });
      // h6 = sum w h5, M = sum w conj(H3c) psi (the 3b2 sources) and the 3b2 field
      if (!pol) {
        K(TC_K_OTHER, fb * (5.0 * P + 4.0), [&] {
          if (bitc)
            hipLaunchKernelGGL((k_reduce_occ<R, N, cx<R>>), dim3(nblk(NR)), dim3(256), 0, s, h5c.p, H3bc.p, psi.p,
                               sh.w.p, P, loc.p + 6 * NR, wk.p);
          else
            hipLaunchKernelGGL((k_reduce_occ<R, N, R>), dim3(nblk(NR)), dim3(256), 0, s, h5.p, H3a4.p, psi.p, sh.w.p,
                               P, loc.p + 6 * NR, wk.p);
        });
        fft3d_t<R, N>(wk.p, 3, -1, s, pf);
        K(TC_K_OTHER, fb * 4.0, [&] {
          hipLaunchKernelGGL((k_gdiv<R, N>), dim3(nblk(NR)), dim3(256), 0, s, rc, tHU.p, wk.p, wk.p + 3 * NR);
        });
        fft3d_t<R, N>(wk.p + 3 * NR, 1, +1, s, pf);
        TC_HIP(hipMemcpyAsync(loc.p + 7 * NR, wk.p + 3 * NR, NR * sizeof(cx<R>), hipMemcpyDeviceToDevice, s));
      } else {
        // per channel M_s2; h6 and the 3b2 field of each target spin from both channels
        for (int s2 = 0; s2 < 2; ++s2)
          K(TC_K_OTHER, fb * (5.0 * P + 4.0), [&] {
            if (bitc)
              hipLaunchKernelGGL((k_reduce_occ<R, N, cx<R>>), dim3(nblk(NR)), dim3(256), 0, s, H5C[s2], HBC[s2],
                                 PSI[s2], W[s2], P, LOC[s2] + 6 * NR, wk2.p + (8 + 3 * s2) * NR);
            else
              hipLaunchKernelGGL((k_reduce_occ<R, N, R>), dim3(nblk(NR)), dim3(256), 0, s, H5P[s2], H3[s2], PSI[s2],
                                 W[s2], P, LOC[s2] + 6 * NR, wk2.p + (8 + 3 * s2) * NR);
          });
        fft3d_t<R, N>(wk2.p + 8 * NR, 6, -1, s, pf);
        for (int sp = 0; sp < 2; ++sp) {
          const int o = 1 - sp;
          K(TC_K_OTHER, fb * (2.0 * P + 1.0), [&] {
            if (bitc)
              hipLaunchKernelGGL((k_h6_pol_c<R, N>), dim3(nblk(NR)), dim3(256), 0, s, H5C[sp], W[sp], H5CA[o], W[o], P,
                                 LOC[sp] + 6 * NR);
            else
              hipLaunchKernelGGL((k_h6_pol<R, N>), dim3(nblk(NR)), dim3(256), 0, s, H5P[sp], W[sp], H5A[o], W[o], P,
                                 LOC[sp] + 6 * NR);
            hipLaunchKernelGGL((k_gdiv2<R, N>), dim3(nblk(NR)), dim3(256), 0, s, rc, tHUp.p, tHUa.p,
                               wk2.p + (8 + 3 * sp) * NR, wk2.p + (8 + 3 * o) * NR, wk.p);
          });
          fft3d_t<R, N>(wk.p, 1, +1, s, pf);
          TC_HIP(hipMemcpyAsync(LOC[sp] + 7 * NR, wk.p, NR * sizeof(cx<R>), hipMemcpyDeviceToDevice, s));
        }
      }
    }
    for (int c = 0; c < ns; ++c)
      K(TC_K_OTHER, 6.0 * fb * P, [&] {
        hipLaunchKernelGGL((k_lattice3<R, N>), dim3(nblk(long(P) * NR)), dim3(256), 0, s, H3[c], HL[c], bm, long(P),
                           3 * NR, NR);
        if (bitc)   // in place: B conj(H3b), the pass-B partner field
          hipLaunchKernelGGL((k_lattice3<R, N>), dim3(nblk(long(P) * NR)), dim3(256), 0, s, HBC[c], HBC[c], bm,
                             long(P), 3 * NR, NR);
      });
    ev.rec(3, s);

    // band divergence corrections: h3 of the band orbitals as rows of the occupied-occupied pass
    // (partners: the mesh orbitals; Delta = k_q - k_b), needed by the band forms of 3a4 and 3b5
    if (ts && ts->OBh4) {
      H3I.alloc(size_t(3) * NTG * NR);
      h5I.alloc(size_t(NTG) * NR);
      for (int a0 = 0; a0 < NTG; a0 += T) {
        const int nt = std::min(T, NTG - a0);
        const long npair = long(nt) * P;
        const FusedArgs fa{P, nt, a0, S, chunk};
        hipLaunchKernelGGL((k_pair_xy<R, N, true>), dim3(unsigned(nt) * N * S), dim3(NTH), 0, s, psiT.p, psi.p, fa,
                           bufA.p);
        zconv<OP_O>(s, npair, a0, miT, tb, 0);
        hipLaunchKernelGGL((k_fused_O<R, N>), dim3(unsigned(nt) * N * S), dim3(NTH), 0, s, bufB.p, psi.p, sh.w.p, fa,
                           miT, rc, dfr.p, h5part.p, H3part.p);
        hipLaunchKernelGGL((k_sum_parts<R, N>), dim3(nblk(long(nt) * NR)), dim3(256), 0, s, 0, S, nt, a0, 0,
                           h5part.p, H3part.p, nullptr, nullptr, h5I.p, H3I.p, nullptr, nullptr);
      }
    }

    // ---- 3/4: target batches of each channel (pass A, pass B, local terms, r -> G); partners of the
    // target's own spin
    for (int c = 0; c < ns; ++c) {
      const int o = pol ? 1 - c : 0;
      if (ts && pol) scatter_targets(c);
      const cx<R>* tP = (ts || sym) ? psiT.p : PSI[c];   // target fields
      const cx<R>* tD = (ts || sym) ? DT.p : DD[c];
      for (int t0 = 0; t0 < NTG; t0 += T) {
        const int nt = std::min(T, NTG - t0);
        const long npair = long(nt) * P;
        TC_HIP(hipMemsetAsync(acc.p, 0, size_t(kAccSlots) * T * NR * sizeof(cx<double>), s));
        TC_HIP(hipMemsetAsync(h4.p, 0, size_t(3) * T * NR * sizeof(cx<R>), s));
        // h4 of the batch's targets (Alg. 3a3): from pass A, or on the h5A path the occupied pass's H3a4 rows
        const cx<R>* h4b = h5A ? H3[c] + size_t(t0) * 3 * NR : h4.p;
        if (!t_arena)
          for (int i = 0; i < 3; ++i) {
            hipEvent_t e;
            TC_HIP(hipEventCreate(&e));
            bev.push_back(e);
          }
        hipEvent_t* be = t_arena ? nullptr : &bev[bev.size() - 3];
        if (be) TC_HIP(hipEventRecord(be[0], s));
        const double part = fb * nt * S;   // one working-precision field per (chunk, target)
        if (need_A) {
          const FusedArgs fa{P, nt, t0, S, chunk};
          // the pairs of the partners q >= Q1 that the store does not hold: bufB [t][P - Q1][5] (the triangular
          // store holds them, reflected, for targets below Q1)
          const bool formA = Q1 < P && (!tri || t0 + nt > Q1);
          if (formA) {
            const int PR = P - Q1;
            const FusedArgs fr{PR, nt, t0, S, (PR + S - 1) / S};
            MeshInfo miR = miT;
            miR.P = PR;
            miR.qoff = Q1;
            const long nprR = long(nt) * PR;
            K(TC_K_XY_PAIR_TGT, fb * (nprR + nt + PR), [&] {
              hipLaunchKernelGGL((k_pair_xy<R, N, false>), dim3(unsigned(nt) * N * S), dim3(NTH), 0, s,
                                 XS[c] + size_t(Q1) * NR, tP, fr, bufA.p);
            });
            K(TC_K_ZCONV_A1, fb * 6.0 * nprR + tabB, [&] {
              zconv<OP_A1>(s, nprR, t0, miR, tb, 1);
            });
          }
          const cx<R>* stp = keepA ? store(c) : nullptr;
          // POL: the antiparallel 3b6 sources take the other channel's density; CN: complex densities
          const cx<R>* nA = pol ? NJ[o] : nullptr;
          const int do3b6 = int(m.m3b6 != 0);
          K(TC_K_FUSED_A, fb * ((m.m3b6 ? 9.0 : 5.0) * npair + 8.0 * P + nt) + (h5A ? 3.5 : 6.0) * part, [&] {
            const dim3 g(unsigned(nt) * N * S), b(NTH);
            if (pol && bitc)
              hipLaunchKernelGGL((k_fused_A<R, N, true, true>), g, b, 0, s, bufB.p, PSI[c], DL[c], HL[c], NJ[c], W[c], fa,
                                 m, do3b6, miT, bm, mm, dfr.p, bufA.p, gpart.p, h4part.p, nA, stp, Q1, int(tri), int(formA));
            else if (pol && h5A)
              hipLaunchKernelGGL((k_fused_A<R, N, true, false, true>), g, b, 0, s, bufB.p, PSI[c], DL[c], HL[c], NJ[c],
                                 W[c], fa, m, do3b6, miT, bm, mm, dfr.p, bufA.p, gpart.p, h4part.p, nA, stp, Q1, int(tri),
                                 int(formA), h5part.p);
            else if (pol)
              hipLaunchKernelGGL((k_fused_A<R, N, true, false>), g, b, 0, s, bufB.p, PSI[c], DL[c], HL[c], NJ[c], W[c], fa,
                                 m, do3b6, miT, bm, mm, dfr.p, bufA.p, gpart.p, h4part.p, nA, stp, Q1, int(tri), int(formA));
            else if (bitc)
              hipLaunchKernelGGL((k_fused_A<R, N, false, true>), g, b, 0, s, bufB.p, PSI[c], DL[c], HL[c], NJ[c], W[c], fa,
                                 m, do3b6, miT, bm, mm, dfr.p, bufA.p, gpart.p, h4part.p, nA, stp, Q1, int(tri), int(formA));
            else if (h5A)
              hipLaunchKernelGGL((k_fused_A<R, N, false, false, true>), g, b, 0, s, bufB.p, PSI[c], DL[c], HL[c], NJ[c],
                                 W[c], fa, m, do3b6, miT, bm, mm, dfr.p, bufA.p, gpart.p, h4part.p, nA, stp, Q1, int(tri),
                                 int(formA), h5part.p);
            else
              hipLaunchKernelGGL((k_fused_A<R, N, false, false>), g, b, 0, s, bufB.p, PSI[c], DL[c], HL[c], NJ[c], W[c],
                                 fa, m, do3b6, miT, bm, mm, dfr.p, bufA.p, gpart.p, h4part.p, nA, stp, Q1, int(tri), int(formA));
          });
          if (h5A)   // h5 (with two channels its parallel part; the antiparallel part in the second half)
            K(TC_K_SUM_PARTS, (pol ? 1.0 : 0.5) * fb * nt * (S + 1), [&] {
              hipLaunchKernelGGL((k_sum_real_parts<R, N>), dim3(nblk(long(nt) * NR)), dim3(256), 0, s, S, nt, t0,
                                 h5part.p, H5P[c]);
              if (pol)
                hipLaunchKernelGGL((k_sum_real_parts<R, N>), dim3(nblk(long(nt) * NR)), dim3(256), 0, s, S, nt, t0,
                                   h5part.p + size_t(S) * nt * NR, H5A[c]);
            });
          K(TC_K_SUM_PARTS, 6.0 * part + 6.0 * fd * nt + 3.0 * fb * nt, [&] {
            hipLaunchKernelGGL((k_sum_parts<R, N>), dim3(nblk(long(nt) * NR)), dim3(256), 0, s, 1, S, nt, t0, 0,
                               nullptr, nullptr, gpart.p, h5A ? nullptr : h4part.p, nullptr, nullptr, acc.p, h4.p);
          });
          if (ts && ts->bdh4) {   // band k-points: h4 of Alg. 3a3 (h3 of Alg. 3b4) corrected at q1 -> k, then <psi_mu|h4_j>
            hipLaunchKernelGGL((k_band_dh4<R, N>), dim3(nblk(long(nt) * NR)), dim3(256), 0, s, tP, ts->bdh4, ts->bV,
                               t0, nt, nbt, h4.p);
            hipLaunchKernelGGL((k_band_dot<R, R, R>), dim3(nt * nbt * 3), dim3(256), 0, s, tP, NR, 0L, h4.p, 3 * NR,
                               NR, t0, (const cx<R>*)nullptr, 0L, t0, nbt, 3, NR, ts->OBh4);
          }
          if (m.m3b6 && !need_B) {
            K(TC_K_ZCONV_A2, fb * 5.0 * npair + tabB, [&] {
              zconv<OP_A2>(s, npair, t0, miT, tb, 1);
            });
            K(TC_K_FUSED_Y, fb * (npair + P) + part, [&] {
              hipLaunchKernelGGL((k_fused_Y<R, N>), dim3(unsigned(nt) * N * S), dim3(NTH), 0, s, bufB.p, PSI[c],
                                 W[c], fa, 1.0, gpart.p);
            });
            K(TC_K_SUM_PARTS, part + 2.0 * fd * nt, [&] {
              hipLaunchKernelGGL((k_sum_parts<R, N>), dim3(nblk(long(nt) * NR)), dim3(256), 0, s, 2, S, nt, t0, 2,
                                 nullptr, nullptr, gpart.p, nullptr, nullptr, nullptr, acc.p, nullptr);
            });
          }
        }
        if (be) TC_HIP(hipEventRecord(be[1], s));
        if (need_B) {
          // With 3b6 selected, its z stage (Alg. 3b6, sources in bufA) and pass B's (Algs. 3b3-3b5, sources in
          // bufB) both multiply by the parallel-channel u~ and end in the same partner sum: one OP_A2 z stage
          // also takes the pass-B sources (with -u~_par: OP_A2 carries -i where pass B carries +i), and one
          // partner sum serves both (three-body energy slot of pass B).
          const bool merged = need_A && m.m3b6;
          const FusedArgs fy{P, nt, t0, S, chunk};
          cx<R>* srcB = merged ? bufB.p : bufA.p;
          cx<R>* zout = merged ? bufB.p + size_t(2) * npair * NR : bufB.p;
          K(TC_K_OTHER, fb * 13.0 * nt, [&] {
            hipLaunchKernelGGL((k_passB_Z<R, N>), dim3(nblk(long(nt) * NR)), dim3(256), 0, s, tP, tD, LOC[c] + NR,
                               h4b, t0, nt, NTG, m, bm, Z.p);
          });
          K(TC_K_XY_PASSB, fb * (2.0 * npair + 4.0 * P + 4.0 * nt), [&] {
            hipLaunchKernelGGL((k_passB_xy<R, N>), dim3(unsigned(nt) * N * S), dim3(NTH), 0, s, tP, XS[c], Z.p,
                               bitc ? HBC[c] : HL[c], fy, miT, dfr.p, R(m.m3b5), srcB);
          });
          if (merged) {
            K(TC_K_ZCONV_A2, fb * 7.0 * npair + tabB, [&] {
              zconv<OP_A2>(s, bufA.p, zout, npair, t0, miT, tb, 1, bufB.p);
            });
          } else {
            K(TC_K_ZCONV_B, fb * 3.0 * npair + tabB, [&] {
              zconv<OP_B>(s, npair, t0, miT, tb, 1);
            });
          }
          K(TC_K_FUSED_Y, fb * (npair + P) + part, [&] {
            hipLaunchKernelGGL((k_fused_Y<R, N>), dim3(unsigned(nt) * N * S), dim3(NTH), 0, s, zout, PSI[c], W[c], fy,
                               1.0, gpart.p);
          });
          K(TC_K_SUM_PARTS, part + 2.0 * fd * nt, [&] {
            hipLaunchKernelGGL((k_sum_parts<R, N>), dim3(nblk(long(nt) * NR)), dim3(256), 0, s, 2, S, nt, t0, 3,
                               nullptr, nullptr, gpart.p, nullptr, nullptr, nullptr, acc.p, nullptr);
          });
        }
        if (be) TC_HIP(hipEventRecord(be[2], s));
        K(TC_K_OTHER, fb * 16.0 * nt + 8.0 * fd * nt, [&] {
          hipLaunchKernelGGL((k_local<R, N>), dim3(nblk(long(nt) * NR)), dim3(256), 0, s, tP, tD, LOC[c], h4b, t0, nt,
                             NTG, m, acc.p, g.p);
          if (!ts)
            hipLaunchKernelGGL((k_epart<R, N>), dim3(kAccSlots * nt), dim3(256), 0, s, sym ? psiT.p : XS[c], acc.p, t0,
                               nt, sym ? sh.epartI.p : sh.epart.p + size_t(kAccSlots) * c * P);
        });
        fft3d_t<R, N>(g.p, nt, -1, s, pf);
        K(TC_K_OTHER, 0.0, [&] {
          hipLaunchKernelGGL((k_gather<R>), dim3(nblk(long(nt) * tnpm)), dim3(256), 0, s, g.p, tbox, tnpw, nbt, tnpm,
                             t0, nt, 1.0 / double(NR),
                             (ts ? ts->out + c * tcofs : sym ? sh.outI.p : sh.out.p + c * cofs), NR,
                             sym ? sh.irrk.p : nullptr);
        });
      }
    }
    if (h5A) {   // the local 3a2 term with h6 from pass A: h6 psi_j, r -> G, added to each target's output
      for (int sp = 0; sp < ns; ++sp) {
        // h6 of spin sp: its own rows' h5 (with two channels the parallel part, and the other spin's rows'
        // antiparallel part)
        cx<R>* h6 = LOC[sp] + 6 * NR;
        const int o = 1 - sp;
        K(TC_K_OTHER, fb * (pol ? 1.0 : 0.5) * P + fb, [&] {
          if (pol)
            hipLaunchKernelGGL((k_h6_pol<R, N>), dim3(nblk(NR)), dim3(256), 0, s, H5P[sp], W[sp], H5A[o], W[o], P, h6);
          else
            hipLaunchKernelGGL((k_h6_sum<R, N>), dim3(nblk(NR)), dim3(256), 0, s, H5P[0], W[0], P, h6);
        });
        K(TC_K_OTHER, fb * (NTG + 1.0), [&] {   // one work-group per target
          hipLaunchKernelGGL((k_h6_energy<R, N>), dim3(NTG), dim3(256), 0, s, XS[sp], h6, 0, 0.5 * m.m3a2, 2,
                             sh.epart.p + size_t(kAccSlots) * sp * P);
        });
        for (int t0 = 0; t0 < NTG; t0 += T) {
          const int nt = std::min(T, NTG - t0);
          K(TC_K_OTHER, fb * (2.0 * nt + 1.0), [&] {
            hipLaunchKernelGGL((k_h6_apply<R, N>), dim3(nblk(long(nt) * NR)), dim3(256), 0, s, PSI[sp], h6, t0, nt,
                               R(0.5 * m.m3a2), g.p);
          });
          fft3d_t<R, N>(g.p, nt, -1, s, pf);
          K(TC_K_OTHER, 0.0, [&] {
            hipLaunchKernelGGL((k_gather<R>), dim3(nblk(long(nt) * tnpm)), dim3(256), 0, s, g.p, tbox, tnpw, nbt, tnpm,
                               t0, nt, 1.0 / double(NR), sh.out.p + sp * cofs, NR, nullptr, 1);
          });
        }
      }
    }
    if (ts && ts->OBh4) band_grid(s, sh, pb, *ts, NTG, psiT.p, tbox, tnpw, tkg, tnpm, rc);
    if (sym)   // every orbital's output and energy slots from its representative's
      K(TC_K_OTHER, 0.0, [&] {
        hipLaunchKernelGGL(k_sym_coef, dim3(nblk(long(P) * pb.npw_max)), dim3(256), 0, s, sh.symk.p, sh.symg0.p,
                           sh.symph.p, sh.npw.p, pb.nk, nb, pb.npw_max, sh.outI.p, sh.out.p);
        hipLaunchKernelGGL(k_sym_epart, dim3(nblk(long(P) * kAccSlots)), dim3(256), 0, s, sh.symk.p, nb, P, kAccSlots,
                           sh.epartI.p, sh.epart.p);
      });
    ev.rec(4, s);

    // ---- 5: kinetic energy and FP64 corrections
    K(TC_K_CORR, 0.0, [&] {
      if (!ts) {
        for (int c = 0; c < ns; ++c)
          hipLaunchKernelGGL(k_kinetic, dim3(P), dim3(256), 0, s, (bitc ? sh.coefL.p : sh.coef.p) + c * cofs,
                             sh.coef.p + c * cofs, sh.kg.p, sh.npw.p, nb, pb.npw_max, sh.tkin.p + size_t(c) * P);
        TC_HIP(hipMemsetAsync(sh.ecorr.p, 0, size_t(2) * ns * P * sizeof(double), s));
      }
      if (need_corr(pb, m) && !(ts && ts->band)) {
        if (pol)
          corrections_pol(s, sh, pb, m, ts);
        else
          corrections(s, sh, pb, m, ts);
      }
    });
    ev.rec(5, s);
    ev.sync(5, s);
    if (pf && pf->on) pf->collect();
    double msA = 0, msB = 0;
    for (size_t i = 0; i + 2 < bev.size(); i += 3) {
      float a = 0, b = 0;
      TC_HIP(hipEventElapsedTime(&a, bev[i], bev[i + 1]));
      TC_HIP(hipEventElapsedTime(&b, bev[i + 1], bev[i + 2]));
      msA += a;
      msB += b;
    }
    for (auto e : bev) (void)hipEventDestroy(e);
    stage_ms[0] = ev.ms(0, 1);
    stage_ms[1] = ev.ms(1, 2);
    stage_ms[2] = ev.ms(2, 3);
    stage_ms[3] = msA;
    stage_ms[4] = msB;
    stage_ms[5] = ev.ms(3, 5) - msA - msB;
  }

  // Grid pieces of the band corrections (see band.hpp and do_apply_band): <psi_mu|psi_j h1>, <H3B_mu|psi_j>,
  // (V . H3B_j)(G); in FP64 the 3a2 field F2 of the occupied set applied to the band orbitals and the 3b6
  // band field with its products and means.
  void band_grid(hipStream_t s, Shared& sh, const Problem& pb, const TargetSet& ts, int NTG, const cx<R>* tP,
                 const int* tbox, const int* tnpw, const double* tkg, int tnpm, const Recip& rc) {
    const int nb = ts.nvec, nkb = ts.nblk, P = pb.P(), nk = pb.nk, npm = pb.npw_max;
    // 3b3: <psi_mu | psi_j h1_c> (h1: Cartesian, loc + N^3)
    hipLaunchKernelGGL((k_band_dot<R, R, R>), dim3(NTG * nb * 3), dim3(256), 0, s, tP, NR, 0L, tP, NR, 0L, 0,
                       (const cx<R>*)(loc.p + NR), NR, 0, nb, 3, NR, ts.OB3);
    // 3b5: <H3B_mu,c | psi_j>; 3a4: (V . H3B_j)(G)
    hipLaunchKernelGGL((k_band_dot<R, R, R>), dim3(NTG * nb * 3), dim3(256), 0, s, H3I.p, 3 * NR, NR, tP, NR, 0L, 0,
                       (const cx<R>*)nullptr, 0L, 0, nb, 3, NR, ts.Z5);
    g.alloc(size_t(std::max(T, NTG)) * NR);
    hipLaunchKernelGGL((k_band_vdot<R, N>), dim3(nblk(long(NTG) * NR)), dim3(256), 0, s, H3I.p, ts.bV, NTG, nb, g.p);
    fft3d_t<R, N>(g.p, NTG, -1, s);
    hipLaunchKernelGGL((k_gather<R>), dim3(nblk(long(NTG) * tnpm)), dim3(256), 0, s, g.p, tbox, tnpw, nb, tnpm, 0, NTG,
                       1.0 / double(NR), ts.W4, NR);
    // FP64: mesh orbitals, n~, the Y source and F2 of 3a2 (as in corrections())
    TC_HIP(hipMemsetAsync(psi64.p, 0, size_t(P) * NR * sizeof(cx<double>), s));
    hipLaunchKernelGGL((k_scatter<double>), dim3(nblk(long(P) * npm)), dim3(256), 0, s, sh.coef.p, sh.boxidx.p,
                       sh.npw.p, sh.kg.p, pb.nb, npm, P, -1, psi64.p, NR);
    fft3d_t<double, N>(psi64.p, P, +1, s);
    hipLaunchKernelGGL(k_overlap, dim3(nk * pb.nb * pb.nb), dim3(256), 0, s, sh.coef.p, pb.nb, sh.coef.p, pb.nb,
                       sh.npw.p, npm, nk, sh.S.p);
    std::vector<double> fo(pb.occ);
    focc.alloc(P);
    TC_HIP(hipMemcpyAsync(focc.p, fo.data(), P * sizeof(double), hipMemcpyHostToDevice, s));
    cx<double>* nG = v64.p;
    cx<double>* YG = v64.p + NR;
    cx<double>* F2 = v64.p + 2 * NR;
    cx<double>* F6 = v64.p + 3 * NR;
    hipLaunchKernelGGL((k_density64<N>), dim3(nblk(NR)), dim3(256), 0, s, psi64.p, psi64.p, sh.w.p, P, nG);
    hipLaunchKernelGGL((k_corr_Ysrc<N>), dim3(nblk(NR)), dim3(256), 0, s, psi64.p, psi64.p, sh.S.p, focc.p, nk, pb.nb,
                       1.0 / (nk * pb.omega), YG);
    fft3d_t<double, N>(nG, 2, -1, s);
    const double a0 = 2 * kPi * corrA[0] / nk, a1 = 2 * kPi * corrA[1] / nk;
    hipLaunchKernelGGL((k_corr_gfields<N>), dim3(nblk(NR)), dim3(256), 0, s, tHu0.p, tHu1.p, 2 * a0, 2 * a1, YG, F2);
    fft3d_t<double, N>(F2, 1, +1, s);
    // band orbitals in FP64
    psiT64.alloc(size_t(NTG) * NR);
    prodT.alloc(size_t(2) * NTG * NR);
    TC_HIP(hipMemsetAsync(psiT64.p, 0, size_t(NTG) * NR * sizeof(cx<double>), s));
    hipLaunchKernelGGL((k_scatter<double>), dim3(nblk(long(NTG) * tnpm)), dim3(256), 0, s, ts.coef, tbox, tnpw, tkg,
                       nb, tnpm, NTG, -1, psiT64.p, NR);
    fft3d_t<double, N>(psiT64.p, NTG, +1, s);
    // 3a2 on the band targets: (F2 psi_j)(G)
    hipLaunchKernelGGL((k_band_mul<N>), dim3(nblk(long(NTG) * NR)), dim3(256), 0, s, F2, psiT64.p, NTG, prodT.p);
    fft3d_t<double, N>(prodT.p, NTG, -1, s);
    hipLaunchKernelGGL((k_gather<double>), dim3(nblk(long(NTG) * tnpm)), dim3(256), 0, s, prodT.p, tbox, tnpw, nb,
                       tnpm, 0, NTG, 1.0 / double(NR), ts.Wa, NR);
    // 3b6 band field of each band k-point, its products with the band orbitals and the means
    for (int b = 0; b < nkb; ++b) {
      hipLaunchKernelGGL((k_band_f3b6<N>), dim3(nblk(NR)), dim3(256), 0, s, rc, tHu0.p, tHu1.p, ts.c3b6[0], ts.c3b6[1],
                         ts.bV + 3 * b, nG, F6);
      fft3d_t<double, N>(F6, 1, +1, s);
      hipLaunchKernelGGL((k_band_mul<N>), dim3(nblk(long(nb) * NR)), dim3(256), 0, s, F6, psiT64.p + size_t(b) * nb * NR,
                         nb, prodT.p + size_t(b) * nb * NR);
      hipLaunchKernelGGL((k_band_dot<double, double, double>), dim3(nb * nb), dim3(256), 0, s, psiT64.p, NR, 0L,
                         prodT.p, NR, 0L, 0, (const cx<double>*)nullptr, 0L, b * nb, nb, 1, NR, ts.OB6);
    }
    fft3d_t<double, N>(prodT.p, NTG, -1, s);
    hipLaunchKernelGGL((k_gather<double>), dim3(nblk(long(NTG) * tnpm)), dim3(256), 0, s, prodT.p, tbox, tnpw, nb,
                       tnpm, 0, NTG, 1.0 / double(NR), ts.X6, NR);
  }

  // Spin-polarised SCF-mesh corrections (FP64): for target spin sp, 2ax with its own channel's overlaps;
  // 3a2 summed over the partner channel s2 with A_{pair(sp, s2)} (Eqs. divcor_3a2_first/second); 3b6
  // summed over the density channel s1 with A_{pair(s1, sp)} (Eqs. 3b6_div_scf1-3).  With identical
  // channels this is the unpolarised form.
  // With a target set: the occupied-set quantities as above, and per channel the target-dependent ones
  // (S(mu, v) = <c_mu|v>, O(mu, v) = <c_mu|F1 v>, W_v = FT(F2 v)) from that channel's trial vectors.
  void corrections_pol(hipStream_t s, Shared& sh, const Problem& pb, const Masks& m, const TargetSet* ts = nullptr) {
    const int P = pb.P(), nb = pb.nb, nk = pb.nk, npm = pb.npw_max;
    const size_t cofs = size_t(2) * P * npm;
    cx<double>* PS64[2] = {psi64.p, psi64_1.p};
    // biorthogonal mode: overlaps S(a,b) = <chi_a|psi_b>, densities and 3a2 sources with conj(chi), energies
    // with <chi| (each channel with its own left set)
    const bool bitc = pb.bitc;
    cx<double>* CH64[2] = {chi64.p, chi64_1.p};
    const cx<double>* X64[2] = {bitc ? chi64.p : psi64.p, bitc ? chi64_1.p : psi64_1.p};
    const double* CL[2] = {(bitc ? sh.coefL.p : sh.coef.p), (bitc ? sh.coefL.p : sh.coef.p) + cofs};
    // per channel: overlaps, FP64 fields, n~ and Y~ (v64p: [0,1] n~, [2,3] Y~, [4] F1, [5] F2)
    sh.S.alloc(size_t(4) * nk * nb * nb);
    std::vector<double> Sh(size_t(4) * nk * nb * nb);
    std::vector<double> focc2(size_t(2) * P);
    for (int p = 0; p < P; ++p) {
      focc2[p] = pb.occ[p];
      focc2[P + p] = pb.occ_dn[p];
    }
    focc.alloc(size_t(2) * P);
    TC_HIP(hipMemcpyAsync(focc.p, focc2.data(), focc2.size() * sizeof(double), hipMemcpyHostToDevice, s));
    for (int sp = 0; sp < 2; ++sp) {
      const double* cf = sh.coef.p + sp * cofs;
      double* Ssp = sh.S.p + size_t(2) * sp * nk * nb * nb;
      hipLaunchKernelGGL(k_overlap, dim3(nk * nb * nb), dim3(256), 0, s, CL[sp], nb, cf, nb, sh.npw.p, npm, nk, Ssp);
      TC_HIP(hipMemsetAsync(PS64[sp], 0, size_t(P) * NR * sizeof(cx<double>), s));
      hipLaunchKernelGGL((k_scatter<double>), dim3(nblk(long(P) * npm)), dim3(256), 0, s, cf, sh.boxidx.p, sh.npw.p,
                         sh.kg.p, nb, npm, P, -1, PS64[sp], NR);
      fft3d_t<double, N>(PS64[sp], P, +1, s);
      if (bitc) {
        TC_HIP(hipMemsetAsync(CH64[sp], 0, size_t(P) * NR * sizeof(cx<double>), s));
        hipLaunchKernelGGL((k_scatter<double>), dim3(nblk(long(P) * npm)), dim3(256), 0, s, CL[sp], sh.boxidx.p,
                           sh.npw.p, sh.kg.p, nb, npm, P, -1, CH64[sp], NR);
        fft3d_t<double, N>(CH64[sp], P, +1, s);
      }
      hipLaunchKernelGGL((k_density64<N>), dim3(nblk(NR)), dim3(256), 0, s, X64[sp], PS64[sp], sh.w.p + sp * P, P,
                         v64p.p + sp * NR);
      hipLaunchKernelGGL((k_corr_Ysrc<N>), dim3(nblk(NR)), dim3(256), 0, s, X64[sp], PS64[sp], Ssp, focc.p + sp * P,
                         nk, nb, 1.0 / (nk * pb.omega), v64p.p + (2 + sp) * NR);
    }
    fft3d_t<double, N>(v64p.p, 4, -1, s);
    TC_HIP(hipMemcpyAsync(Sh.data(), sh.S.p, Sh.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    // per channel: n~(0) and sum_ab f_a f_b S(a,b) S(b,a) / Omega^2 (real in TC mode, complex in the
    // biorthogonal mode: imaginary parts n0i, csi)
    double n0[2] = {0, 0}, cs[2] = {0, 0}, n0i[2] = {0, 0}, csi[2] = {0, 0};
    for (int sp = 0; sp < 2; ++sp) {
      const double* S = &Sh[size_t(2) * sp * nk * nb * nb];
      const double* f = sp == 0 ? pb.occ.data() : pb.occ_dn.data();
      for (int k = 0; k < nk; ++k)
        for (int a = 0; a < nb; ++a) {
          n0[sp] += f[k * nb + a] / nk * S[2 * ((k * nb + a) * nb + a)] / pb.omega;
          n0i[sp] += f[k * nb + a] / nk * S[2 * ((k * nb + a) * nb + a) + 1] / pb.omega;
          for (int b = 0; b < nb; ++b) {
            const double* sab = &S[2 * ((k * nb + a) * nb + b)];
            const double* sba = &S[2 * ((k * nb + b) * nb + a)];
            const double fab = f[k * nb + a] / nk * f[k * nb + b] / (pb.omega * pb.omega);
            cs[sp] += fab * (sab[0] * sba[0] - sab[1] * sba[1]);
            csi[sp] += fab * (sab[0] * sba[1] + sab[1] * sba[0]);
          }
        }
    }
    const double a0 = 2 * kPi * corrA[0] / nk, a1 = 2 * kPi * corrA[1] / nk;
    for (int sp = 0; sp < 2; ++sp) {
      const int o = 1 - sp;
      const double* cf = sh.coef.p + sp * cofs;
      const double* Ssp = sh.S.p + size_t(2) * sp * nk * nb * nb;
      cx<double>* F1 = v64p.p + 4 * NR;
      cx<double>* F2 = v64p.p + 5 * NR;
      hipLaunchKernelGGL((k_corr_gfields2<N>), dim3(nblk(NR)), dim3(256), 0, s, tHu0.p, tHu1.p, a0, a1,
                         v64p.p + sp * NR, v64p.p + o * NR, F1);
      hipLaunchKernelGGL((k_corr_gfields2<N>), dim3(nblk(NR)), dim3(256), 0, s, tHu0.p, tHu1.p, 2 * a0, 2 * a1,
                         v64p.p + (2 + sp) * NR, v64p.p + (2 + o) * NR, F2);
      fft3d_t<double, N>(F1, 2, +1, s);
      hipLaunchKernelGGL((k_corr_products<N>), dim3(nblk(2L * P * NR)), dim3(256), 0, s, F1, PS64[sp], P, prod64.p);
      fft3d_t<double, N>(prod64.p, 2L * P, -1, s);
      double* Zg = sh.Zg.p + sp * cofs;
      double* Wg = sh.Wg.p + sp * cofs;
      hipLaunchKernelGGL((k_gather<double>), dim3(nblk(long(P) * npm)), dim3(256), 0, s, prod64.p, sh.boxidx.p,
                         sh.npw.p, nb, npm, 0, P, 1.0 / double(NR), Zg, NR);
      hipLaunchKernelGGL((k_gather<double>), dim3(nblk(long(P) * npm)), dim3(256), 0, s, prod64.p + size_t(P) * NR,
                         sh.boxidx.p, sh.npw.p, nb, npm, 0, P, 1.0 / double(NR), Wg, NR);
      hipLaunchKernelGGL(k_overlap, dim3(nk * nb * nb), dim3(256), 0, s, CL[sp], nb, Zg, nb, sh.npw.p, npm, nk, sh.O.p);
      // channel prefactors: pair(sp, sp) = parallel, pair(sp, o) = antiparallel
      const double c1a_p = kFourPi * corrB[0], c1a_a = kFourPi * corrB[1];
      const double c1s_p = 2 * kPi * corrB[0], c1s_a = 2 * kPi * corrB[1];
      const double const1 = c1a_p * cs[sp] + c1a_a * cs[o], const1i = c1a_p * csi[sp] + c1a_a * csi[o];
      const double c1sn0 = c1s_p * n0[sp] + c1s_a * n0[o], c1sn0i = c1s_p * n0i[sp] + c1s_a * n0i[o];
      if (!ts) {
        hipLaunchKernelGGL(k_corr_apply, dim3(nblk(long(P) * npm)), dim3(256), 0, s, cf, cf, Ssp, sh.O.p, Zg, Wg,
                           focc.p + sp * P, sh.npw.p, nb, nb, npm, P, pb.omega, 1.0, dgb_eff(pb, m, corrA[0]), m.m3a2,
                           const1, const1i, m.m3b6, c1sn0, c1sn0i, sh.dhc2.p + sp * cofs, sh.dhc3.p + sp * cofs);
        hipLaunchKernelGGL(k_corr_add, dim3(P), dim3(256), 0, s, CL[sp], sh.dhc2.p + sp * cofs, sh.dhc3.p + sp * cofs,
                           sh.npw.p, nb, npm, sh.out.p + sp * cofs, sh.ecorr.p + size_t(2) * sp * P);
        continue;
      }
      // this channel's trial vectors as targets
      const int nv = ts->nvec, NT = nk * nv;
      const size_t nc = size_t(2) * NT * npm;
      const double* tcf = ts->coef + sp * nc;
      psiT64.alloc(size_t(NT) * NR);
      prodT.alloc(size_t(2) * NT * NR);
      for (auto* b : {&sh.ZgT, &sh.WgT, &sh.dhc2T, &sh.dhc3T}) b->alloc(nc);
      sh.ST.alloc(size_t(2) * nk * nb * nv);
      sh.OT.alloc(size_t(2) * nk * nb * nv);
      sh.ecorrT.alloc(size_t(2) * NT);
      TC_HIP(hipMemsetAsync(psiT64.p, 0, size_t(NT) * NR * sizeof(cx<double>), s));
      hipLaunchKernelGGL((k_scatter<double>), dim3(nblk(long(NT) * npm)), dim3(256), 0, s, tcf, sh.boxidx.p, sh.npw.p,
                         sh.kg.p, nv, npm, NT, -1, psiT64.p, NR);
      fft3d_t<double, N>(psiT64.p, NT, +1, s);
      hipLaunchKernelGGL((k_corr_products<N>), dim3(nblk(2L * NT * NR)), dim3(256), 0, s, F1, psiT64.p, NT, prodT.p);
      fft3d_t<double, N>(prodT.p, 2L * NT, -1, s);
      hipLaunchKernelGGL((k_gather<double>), dim3(nblk(long(NT) * npm)), dim3(256), 0, s, prodT.p, sh.boxidx.p,
                         sh.npw.p, nv, npm, 0, NT, 1.0 / double(NR), sh.ZgT.p, NR);
      hipLaunchKernelGGL((k_gather<double>), dim3(nblk(long(NT) * npm)), dim3(256), 0, s, prodT.p + size_t(NT) * NR,
                         sh.boxidx.p, sh.npw.p, nv, npm, 0, NT, 1.0 / double(NR), sh.WgT.p, NR);
      hipLaunchKernelGGL(k_overlap, dim3(nk * nb * nv), dim3(256), 0, s, CL[sp], nb, tcf, nv, sh.npw.p, npm, nk,
                         sh.ST.p);
      hipLaunchKernelGGL(k_overlap, dim3(nk * nb * nv), dim3(256), 0, s, CL[sp], nb, sh.ZgT.p, nv, sh.npw.p, npm, nk,
                         sh.OT.p);
      hipLaunchKernelGGL(k_corr_apply, dim3(nblk(long(NT) * npm)), dim3(256), 0, s, tcf, cf, sh.ST.p, sh.OT.p, Zg,
                         sh.WgT.p, focc.p + sp * P, sh.npw.p, nb, nv, npm, NT, pb.omega, 1.0,
                         dgb_eff(pb, m, corrA[0]), m.m3a2, const1, const1i, m.m3b6, c1sn0, c1sn0i, sh.dhc2T.p,
                         sh.dhc3T.p);
      hipLaunchKernelGGL(k_corr_add, dim3(NT), dim3(256), 0, s, tcf, sh.dhc2T.p, sh.dhc3T.p, sh.npw.p, nv, npm,
                         ts->out + sp * nc, sh.ecorrT.p);
    }
  }

  // SCF-mesh divergence corrections in FP64 (2ax, 3a2, 3b6); see k_corr_apply.
  // Biorthogonal mode: overlaps S(a,b) = <chi_a|psi_b>, densities and 3a2 sources with conj(chi),
  // energies with <chi|.
  // With a target set, the occupied-set quantities are formed the same way and the target-dependent ones
  // (S(mu, v) = <chi_mu|v>, O(mu, v) = <chi_mu|F1 v>, W_v = FT(F2 v)) from the trial vectors.
  void corrections(hipStream_t s, Shared& sh, const Problem& pb, const Masks& m, const TargetSet* ts) {
    const int P = pb.P(), nb = pb.nb, nk = pb.nk;
    const bool bitc = pb.bitc;
    const double* cl = bitc ? sh.coefL.p : sh.coef.p;
    hipLaunchKernelGGL(k_overlap, dim3(nk * nb * nb), dim3(256), 0, s, cl, nb, sh.coef.p, nb, sh.npw.p, pb.npw_max,
                       nk, sh.S.p);
    std::vector<double> S(size_t(2) * nk * nb * nb);
    TC_HIP(hipMemcpyAsync(S.data(), sh.S.p, S.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    TC_HIP(hipMemcpyAsync(focc.p, pb.occ.data(), P * sizeof(double), hipMemcpyHostToDevice, s));
    // FP64 orbitals on the grid
    TC_HIP(hipMemsetAsync(psi64.p, 0, size_t(P) * NR * sizeof(cx<double>), s));
    hipLaunchKernelGGL((k_scatter<double>), dim3(nblk(long(P) * pb.npw_max)), dim3(256), 0, s, sh.coef.p, sh.boxidx.p,
                       sh.npw.p, sh.kg.p, nb, pb.npw_max, P, -1, psi64.p, NR);
    fft3d_t<double, N>(psi64.p, P, +1, s);
    if (bitc) {
      TC_HIP(hipMemsetAsync(chi64.p, 0, size_t(P) * NR * sizeof(cx<double>), s));
      hipLaunchKernelGGL((k_scatter<double>), dim3(nblk(long(P) * pb.npw_max)), dim3(256), 0, s, sh.coefL.p,
                         sh.boxidx.p, sh.npw.p, sh.kg.p, nb, pb.npw_max, P, -1, chi64.p, NR);
      fft3d_t<double, N>(chi64.p, P, +1, s);
    }
    const cx<double>* X64 = bitc ? chi64.p : psi64.p;
    cx<double>* nG = v64.p;
    cx<double>* YG = v64.p + NR;
    cx<double>* F1 = v64.p + 2 * NR;
    cx<double>* F2 = v64.p + 3 * NR;
    hipLaunchKernelGGL((k_density64<N>), dim3(nblk(NR)), dim3(256), 0, s, X64, psi64.p, sh.w.p, P, nG);
    hipLaunchKernelGGL((k_corr_Ysrc<N>), dim3(nblk(NR)), dim3(256), 0, s, X64, psi64.p, sh.S.p, focc.p, nk, nb,
                       1.0 / (nk * pb.omega), YG);
    fft3d_t<double, N>(nG, 2, -1, s);
    const double a0 = 2 * kPi * corrA[0] / nk, a1 = 2 * kPi * corrA[1] / nk;
    hipLaunchKernelGGL((k_corr_gfields<N>), dim3(nblk(NR)), dim3(256), 0, s, tHu0.p, tHu1.p, a0, a1, nG, F1);
    hipLaunchKernelGGL((k_corr_gfields<N>), dim3(nblk(NR)), dim3(256), 0, s, tHu0.p, tHu1.p, 2 * a0, 2 * a1, YG, F2);
    fft3d_t<double, N>(F1, 2, +1, s);
    hipLaunchKernelGGL((k_corr_products<N>), dim3(nblk(2L * P * NR)), dim3(256), 0, s, F1, psi64.p, P, prod64.p);
    fft3d_t<double, N>(prod64.p, 2L * P, -1, s);
    hipLaunchKernelGGL((k_gather<double>), dim3(nblk(long(P) * pb.npw_max)), dim3(256), 0, s, prod64.p, sh.boxidx.p,
                       sh.npw.p, nb, pb.npw_max, 0, P, 1.0 / double(NR), sh.Zg.p, NR);
    hipLaunchKernelGGL((k_gather<double>), dim3(nblk(long(P) * pb.npw_max)), dim3(256), 0, s,
                       prod64.p + size_t(P) * NR, sh.boxidx.p, sh.npw.p, nb, pb.npw_max, 0, P, 1.0 / double(NR),
                       sh.Wg.p, NR);
    hipLaunchKernelGGL(k_overlap, dim3(nk * nb * nb), dim3(256), 0, s, cl, nb, sh.Zg.p, nb, sh.npw.p, pb.npw_max,
                       nk, sh.O.p);
    TC_HIP(hipStreamSynchronize(s));
    // scalars: n~(0) per spin and const1 of the G = G' = 0 correction of 3a2
    double n0 = 0, n0i = 0;   // n~(0) = sum_a w_a S(a,a) / Omega (real in TC mode)
    for (int k = 0; k < nk; ++k)
      for (int a = 0; a < nb; ++a) {
        n0 += pb.occ[k * nb + a] / nk * S[2 * ((k * nb + a) * nb + a)] / pb.omega;
        if (bitc) n0i += pb.occ[k * nb + a] / nk * S[2 * ((k * nb + a) * nb + a) + 1] / pb.omega;
      }
    double c1s = 0, c1a = 0;
    for (int ch = 0; ch < 2; ++ch) {
      c1s += 2 * kPi * corrB[ch];   // Eq. 3b6_div_scf1 (summed over the density's spin)
      c1a += kFourPi * corrB[ch];   // Eq. divcor_3a2_first (summed over the partners' spin)
    }
    double const1 = 0, const1i = 0;   // sum f_a f_b S(a,b) S(b,a) (real in TC mode)
    for (int k = 0; k < nk; ++k)
      for (int a = 0; a < nb; ++a)
        for (int b = 0; b < nb; ++b) {
          const double* sab = &S[2 * ((k * nb + a) * nb + b)];
          const double* sba = &S[2 * ((k * nb + b) * nb + a)];
          const double re = sab[0] * sba[0] - sab[1] * sba[1];
          const double fab = pb.occ[k * nb + a] / nk * pb.occ[k * nb + b] * c1a / (pb.omega * pb.omega);
          const1 += fab * re;
          if (bitc) const1i += fab * (sab[0] * sba[1] + sab[1] * sba[0]);
        }
    if (!ts) {
      hipLaunchKernelGGL(k_corr_apply, dim3(nblk(long(P) * pb.npw_max)), dim3(256), 0, s, sh.coef.p, sh.coef.p,
                         sh.S.p, sh.O.p, sh.Zg.p, sh.Wg.p, focc.p, sh.npw.p, nb, nb, pb.npw_max, P, pb.omega, 1.0,
                         dgb_eff(pb, m, corrA[0]), m.m3a2, const1, const1i, m.m3b6, c1s * n0, c1s * n0i, sh.dhc2.p, sh.dhc3.p);
      hipLaunchKernelGGL(k_corr_add, dim3(P), dim3(256), 0, s, cl, sh.dhc2.p, sh.dhc3.p, sh.npw.p, nb, pb.npw_max,
                         sh.out.p, sh.ecorr.p);
      return;
    }
    // target set: FP64 fields of the trial vectors, F1 v and F2 v, overlaps with the left occupied set
    const int nv = ts->nvec, NT = nk * nv;
    const size_t nc = size_t(2) * NT * pb.npw_max;
    psiT64.alloc(size_t(NT) * NR);
    prodT.alloc(size_t(2) * NT * NR);
    sh.ZgT.alloc(nc);
    sh.WgT.alloc(nc);
    sh.dhc2T.alloc(nc);
    sh.dhc3T.alloc(nc);
    sh.ST.alloc(size_t(2) * nk * nb * nv);
    sh.OT.alloc(size_t(2) * nk * nb * nv);
    sh.ecorrT.alloc(size_t(2) * NT);
    TC_HIP(hipMemsetAsync(psiT64.p, 0, size_t(NT) * NR * sizeof(cx<double>), s));
    hipLaunchKernelGGL((k_scatter<double>), dim3(nblk(long(NT) * pb.npw_max)), dim3(256), 0, s, ts->coef, sh.boxidx.p,
                       sh.npw.p, sh.kg.p, nv, pb.npw_max, NT, -1, psiT64.p, NR);
    fft3d_t<double, N>(psiT64.p, NT, +1, s);
    hipLaunchKernelGGL((k_corr_products<N>), dim3(nblk(2L * NT * NR)), dim3(256), 0, s, F1, psiT64.p, NT, prodT.p);
    fft3d_t<double, N>(prodT.p, 2L * NT, -1, s);
    hipLaunchKernelGGL((k_gather<double>), dim3(nblk(long(NT) * pb.npw_max)), dim3(256), 0, s, prodT.p, sh.boxidx.p,
                       sh.npw.p, nv, pb.npw_max, 0, NT, 1.0 / double(NR), sh.ZgT.p, NR);
    hipLaunchKernelGGL((k_gather<double>), dim3(nblk(long(NT) * pb.npw_max)), dim3(256), 0, s,
                       prodT.p + size_t(NT) * NR, sh.boxidx.p, sh.npw.p, nv, pb.npw_max, 0, NT, 1.0 / double(NR),
                       sh.WgT.p, NR);
    hipLaunchKernelGGL(k_overlap, dim3(nk * nb * nv), dim3(256), 0, s, cl, nb, ts->coef, nv, sh.npw.p, pb.npw_max, nk,
                       sh.ST.p);
    hipLaunchKernelGGL(k_overlap, dim3(nk * nb * nv), dim3(256), 0, s, cl, nb, sh.ZgT.p, nv, sh.npw.p, pb.npw_max, nk,
                       sh.OT.p);
    hipLaunchKernelGGL(k_corr_apply, dim3(nblk(long(NT) * pb.npw_max)), dim3(256), 0, s, ts->coef, sh.coef.p, sh.ST.p,
                       sh.OT.p, sh.Zg.p, sh.WgT.p, focc.p, sh.npw.p, nb, nv, pb.npw_max, NT, pb.omega, 1.0,
                       dgb_eff(pb, m, corrA[0]), m.m3a2, const1, const1i, m.m3b6, c1s * n0, c1s * n0i, sh.dhc2T.p, sh.dhc3T.p);
    hipLaunchKernelGGL(k_corr_add, dim3(NT), dim3(256), 0, s, ts->coef, sh.dhc2T.p, sh.dhc3T.p, sh.npw.p, nv,
                       pb.npw_max, ts->out, sh.ecorrT.p);
  }
};

template <typename R, int N>
Engine* new_engine(bool zmfma) {
  auto* e = new EngineT<R, N>();
  e->zmfma = zmfma;
  if (zmfma) e->upload_zfrag();
  return e;
}

template <typename R>
Engine* make_engine_r(int N, bool zmfma = false) {
  switch (N) {
    case 8: return new_engine<R, 8>(zmfma);
#ifndef TCMI_HOST_CHECK_BUILD   // the host sanitizer build of the tests compiles the 8-point engine only
    case 12: return new_engine<R, 12>(zmfma);
    case 16: return new_engine<R, 16>(zmfma);
    case 24: return new_engine<R, 24>(zmfma);
    case 32: return new_engine<R, 32>(zmfma);
    case 48: return new_engine<R, 48>(zmfma);
#endif
    default: return nullptr;
  }
}

void upload_twiddles() {
  static bool done = false;   // per process; constant memory is per device, re-uploaded per context below
  (void)done;
  const int sizes[6] = {8, 12, 16, 24, 32, 48};
  std::vector<double> t64(2 * kTwTotal);
  std::vector<float> t32(2 * kTwTotal);
  for (int N : sizes) {
    const int off = tw_off(N);
    for (int m = 0; m < N; ++m) {
      const double a = -2.0 * kPi * m / N;
      t64[2 * (off + m)] = std::cos(a);
      t64[2 * (off + m) + 1] = std::sin(a);
      t32[2 * (off + m)] = float(std::cos(a));
      t32[2 * (off + m) + 1] = float(std::sin(a));
    }
  }
  TC_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_tw64), t64.data(), t64.size() * sizeof(double)));
  TC_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_tw32), t32.data(), t32.size() * sizeof(float)));
}

}  // namespace

// ====================================================================== C ABI
// Scratch of tc_apply_all_dev_noalloc: every device buffer of that call is carved from it (Arena).  Each
// device that loads the library holds its own copy until the process ends.  Host code reaches it only
// through the address hipGetSymbolAddress returns on each device (scratch_on), never through the name.
constexpr size_t kNoAllocScratchBytes = size_t(256) << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {
std::mutex g_scratch_mu;
std::unordered_map<int, char*> g_scratch;   // device -> address of its scratch

// Address of `scratch` on `device`, which must be the current device; looked up once per device.
char* scratch_on(int device) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  auto it = g_scratch.find(device);
  if (it != g_scratch.end()) return it->second;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr)
    throw TcError(TC_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  g_scratch[device] = static_cast<char*>(ptr);
  return static_cast<char*>(ptr);
}

// For the length of a no-allocation call: device buffers are carved from the scratch (Arena), and
// every buffer rebound or hidden during the call gets its previous state back at the end.
struct ArenaScope {
  Arena arena;
  explicit ArenaScope(char* base) {
    arena.base = base;
    arena.cap = kNoAllocScratchBytes;
    t_arena = &arena;
  }
  ~ArenaScope() {
    t_arena = nullptr;
    for (auto it = arena.undo.rbegin(); it != arena.undo.rend(); ++it) (*it)();
  }
};
}  // namespace

struct tc_ctx {
  // caller allocators (tc_set_allocator), first so that they outlive every buffer they made; entries are
  // never changed, each buffer frees through the one that made it
  std::list<DevAlloc> allocs;
  const DevAlloc* cur_alloc = nullptr;
  char* scratch = nullptr;   // this device's no-allocation scratch (set at tc_create)
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::string err;
  Problem pb;
  Shared sh;
  std::unique_ptr<Engine> eng;
  int eng_prec = -1, eng_N = -1;
  bool tables_dirty = true;
  bool have_result = false;
  std::vector<double> hcoef;   // [P][npw_max] complex staging
  double e_total = 0, e_parts[TC_E_NPARTS] = {0, 0, 0, 0};
  std::vector<double> eps;   // [P] complex orbital energies of the last application
  DBuf<double> coefT, outT;  // host-buffer tc_apply staging
  // block-Davidson self-consistent loop
  DBuf<double> dV, dHV, dHs, dwork, dX, dY, deval, deps, dcur, dold, dnew, dmix, dchange, dkg2;
  DBuf<int> dvalid, dstatus, dnpw2;
  double stage_ms[6] = {0, 0, 0, 0, 0, 0};
  double total_ms = 0;
  Prof prof;
};

namespace {

int fail(tc_ctx* c, int code, const std::string& m) {
  if (c) c->err = m;
  return code;
}

// Device memory of a call comes from the context's allocator (t_alloc) for the length of the call.
struct AllocScope {
  const DevAlloc* prev;
  explicit AllocScope(const DevAlloc* a) : prev(t_alloc) { t_alloc = a; }
  ~AllocScope() { t_alloc = prev; }
};

template <class F>
int guard(tc_ctx* c, F&& f) {
  if (!c) return TC_ERR_ARG;
  try {
    c->err.clear();
    TC_HIP(hipSetDevice(c->device));
    AllocScope as(c->cur_alloc);
    return f();
  } catch (const TcError& e) {
    return fail(c, e.code, e.msg);
  } catch (const std::bad_alloc&) {
    return fail(c, TC_ERR_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(c, TC_ERR_DEVICE, e.what());
  }
}

// Entry points that only describe the problem (no device work): the same error handling, no device
// selection, so that they also run where no device is present (the host sanitizer build of the tests).
template <class F>
int guard_host(tc_ctx* c, F&& f) {
  if (!c) return TC_ERR_ARG;
  try {
    c->err.clear();
    return f();
  } catch (const TcError& e) {
    return fail(c, e.code, e.msg);
  } catch (const std::bad_alloc&) {
    return fail(c, TC_ERR_OOM, "host allocation failed");
  } catch (const std::exception& e) {
    return fail(c, TC_ERR_DEVICE, e.what());
  }
}

bool grid_supported(int N) { return N == 8 || N == 12 || N == 16 || N == 24 || N == 32 || N == 48; }

void upload_basis_data(tc_ctx* c);
int prepare(tc_ctx* c);
void alloc_shared(tc_ctx* c);
// ------------------------------------------------------------------ band (zero-weight) k-points
int set_band_kpoints(tc_ctx* c, int nkb, const double* kfrac) {
  Problem& pb = c->pb;
  if (pb.nk == 0) return fail(c, TC_ERR_STATE, "set the k-mesh before band k-points");
  if (nkb < 0 || nkb > 4096 || (nkb > 0 && !kfrac)) return fail(c, TC_ERR_ARG, "0 <= nkb <= 4096 and k-points needed");
  pb.nkb = nkb;
  pb.bk.assign(kfrac, kfrac + 3 * size_t(nkb));
  pb.bmiller.assign(nkb, {});
  pb.bnpw.assign(nkb, 0);
  pb.bnb = 0;
  pb.bocc.clear();
  pb.bloaded.assign(nkb, 0);
  pb.band_alpha = -1;
  c->tables_dirty = true;   // band shift tables
  return TC_OK;
}

int set_band_basis(tc_ctx* c, int ib, int npw, const int32_t* miller) {
  Problem& pb = c->pb;
  if (pb.N == 0) return fail(c, TC_ERR_STATE, "set the grid first");
  if (ib < 0 || ib >= pb.nkb || npw <= 0 || !miller) return fail(c, TC_ERR_ARG, "bad band basis arguments");
  for (int g = 0; g < 3 * npw; ++g)
    if (miller[g] >= pb.N / 2 || miller[g] < -(pb.N / 2) + 1)
      return fail(c, TC_ERR_GRID, "plane wave outside the FFT grid");
  pb.bmiller[ib].assign(miller, miller + 3 * size_t(npw));
  pb.bnpw[ib] = npw;
  std::fill(pb.bloaded.begin(), pb.bloaded.end(), 0);   // the coefficient layout follows max npw
  return TC_OK;
}

int load_band_orbitals(tc_ctx* c, int ib, int nband, const double* coef, const double* occ) {
  Problem& pb = c->pb;
  Shared& sh = c->sh;
  if (ib < 0 || ib >= pb.nkb) return fail(c, TC_ERR_ARG, "band k-point index out of range");
  for (int b = 0; b < pb.nkb; ++b)
    if (pb.bnpw[b] <= 0) return fail(c, TC_ERR_STATE, "tc_set_band_basis missing for band k-point " + std::to_string(b));
  if (nband <= 0 || !coef || !occ) return fail(c, TC_ERR_ARG, "nband must be positive, coef and occ non-null");
  if (nband > pb.bnpw[ib]) return fail(c, TC_ERR_ARG, "more bands than plane waves");
  for (int b = 0; b < nband; ++b)
    if (!(occ[b] >= 0.0 && occ[b] <= 1.0)) return fail(c, TC_ERR_ARG, "fillings must lie in [0, 1]");
  if (pb.bnb != nband) {
    pb.bnb = nband;
    std::fill(pb.bloaded.begin(), pb.bloaded.end(), 0);
  }
  pb.bocc.resize(size_t(pb.nkb) * nband);
  for (int b = 0; b < nband; ++b) pb.bocc[size_t(ib) * nband + b] = occ[b];
  int mx = 0;
  for (int b = 0; b < pb.nkb; ++b) mx = std::max(mx, pb.bnpw[b]);
  if (mx != sh.bnpm || sh.bcoef.n < size_t(2) * pb.nkb * nband * mx) {
    sh.bcoef.alloc(size_t(2) * pb.nkb * nband * mx);
    std::fill(pb.bloaded.begin(), pb.bloaded.end(), 0);
  }
  sh.bnpm = mx;
  std::vector<double> stage(size_t(2) * nband * mx, 0.0);
  for (int b = 0; b < nband; ++b)
    std::memcpy(&stage[size_t(2) * b * mx], coef + size_t(2) * b * pb.bnpw[ib], size_t(2) * pb.bnpw[ib] * sizeof(double));
  TC_HIP(hipMemcpy(sh.bcoef.p + size_t(2) * ib * nband * mx, stage.data(), stage.size() * sizeof(double),
                   hipMemcpyHostToDevice));
  pb.bloaded[ib] = 1;
  return TC_OK;
}

// GB quantities at band k-point kf (off the mesh, no vanishing argument): Delta_GB^band =
// Omega / (4 sqrt(pi^3 alpha)) - (1/N_k) sum_{q,G} A_aux(k - q + G) (Eq. divcorr_2ax_band, divided by 4 pi)
// and V = (1/N_k) sum_{q,G} (k - q + G) A_aux(k - q + G) (Cartesian; the vector sum of Eq. correction_nabla at
// the arguments of the kernel it replaces).  False when some k - q + G vanishes (k on the mesh).
bool gb_band(const Problem& pb, const double* kf, double& dgb, double* V) {
  const double a = pb.alpha;
  const double qmax = std::sqrt(41.45 / a);
  int mm[3];
  for (int i = 0; i < 3; ++i) {
    const double L = std::sqrt(pb.lat[3 * i] * pb.lat[3 * i] + pb.lat[3 * i + 1] * pb.lat[3 * i + 1] +
                               pb.lat[3 * i + 2] * pb.lat[3 * i + 2]);
    mm[i] = int(std::ceil(qmax * L / (2 * kPi))) + 3;
  }
  double sum = 0, comp = 0, v[3] = {0, 0, 0};
  for (int ik = 0; ik < pb.nk; ++ik) {
    double f[3];
    pb.kfrac(ik, f);
    for (int m1 = -mm[0]; m1 <= mm[0]; ++m1)
      for (int m2 = -mm[1]; m2 <= mm[1]; ++m2)
        for (int m3 = -mm[2]; m3 <= mm[2]; ++m3) {
          const double c1 = m1 + kf[0] - f[0], c2 = m2 + kf[1] - f[1], c3 = m3 + kf[2] - f[2];
          double Q[3];
          for (int cc = 0; cc < 3; ++cc) Q[cc] = c1 * pb.B[cc] + c2 * pb.B[3 + cc] + c3 * pb.B[6 + cc];
          const double q2 = Q[0] * Q[0] + Q[1] * Q[1] + Q[2] * Q[2];
          if (q2 < 1e-16) return false;
          if (a * q2 >= 41.45) continue;
          const double t = std::exp(-a * q2) / q2;
          const double y = t - comp, z = sum + y;   // Kahan
          comp = (z - sum) - y;
          sum = z;
          for (int cc = 0; cc < 3; ++cc) v[cc] += Q[cc] * t;
        }
  }
  dgb = pb.omega / (4.0 * std::sqrt(kPi * kPi * kPi * a)) - sum / pb.nk;
  for (int cc = 0; cc < 3; ++cc) V[cc] = v[cc] / pb.nk;
  return true;
}

// Band forms of the divergence corrections, combined in FP64 on the host (coefficients on each band
// k-point's plane waves; psi = sqrt(Omega) phi, rho~_{mu j}(0) = S_mu,j / Omega; the multiplicities of the
// three-body terms are those of the operator).  Singular exchange sums at Delta = k - q get the GB
// replacement of Eq. correction (Delta_GB^band) or Eq. correction_nabla (V) with the band k-point's own
// orbitals mu (fillings f_mu):
//   2ax  (Eq. divcorr_2ax_band):  -4 pi Dgb sum f rho c_mu
//   2bx1 (Eq. divcorr_2bx1):      -4 pi A sum f rho (V . (k+G)) c_mu
//   2bx2 (Eq. divcorr_2bx2):      -i 4 pi A sum f (V . X_mu,j) c_mu,   X = (i/Omega) sum conj(c_mu)(k+G) c_j
//   3a3, 3b4 (h4 correction, Eqs. divcorr_3a3, div_corr_3b4_2): on the device before pass B
//   3b4  (Eq. div_corr_3b4_4):    2 x -(i/2) 4 pi A sum f (V . <psi_mu|h4_j>/Omega) c_mu
//   3b3  (Eq. div_corr_3b3_2):    2 x (i/2) 4 pi A sum f (V . <psi_mu|psi_j h1>/Omega) c_mu
//   3a4  (Eqs. div_corr_3a4_2/3, reading R14): 2 x [(i/2) 4 pi A sum f rho_mu2,j (V . H3_mu2)(G)
//                                      + (1/2)(4 pi A)^2 V.V sum f f rho_mu1,mu2 rho_mu2,j c_mu1]
//   3b5  (Eqs. 3b5_div_2/3, R14): 2 x [-(i/2) 4 pi A sum f (V . <H3_mu2|psi_j>/Omega) c_mu2
//                                      + (1/2)(4 pi A)^2 V.V sum f f rho_mu2,mu1 rho_mu1,j c_mu2]
//   3b6  (Eqs. 3b6_div_band1-3):  2 x sum f [c1b n0 rho c_mu + rho (F psi_mu)(G) - <psi_mu|F psi_j>/Omega c_mu]
//   3a2  (the corrections of the mesh rows' h5, Eqs. divcor_3a2_first/second): (1/2)(const1 c_j + (F2 psi_j)(G))
void band_corrections_host(tc_ctx* c, const Masks& m, const std::vector<double>& cb,
                           const std::vector<std::complex<double>>& Sb, const std::vector<double>& dgbb,
                           const std::vector<double>& Vb, std::vector<double>& out) {
  using zc = std::complex<double>;
  Problem& pb = c->pb;
  Shared& sh = c->sh;
  const int nkb = pb.nkb, nb = pb.bnb, npm = sh.bnpm, NTG = nkb * nb;
  const double Om = pb.omega, a4 = kFourPi * pb.A[0];
  auto rd = [&](DBuf<double>& d, size_t n) {
    std::vector<double> h(n);
    TC_HIP(hipMemcpy(h.data(), d.p, n * sizeof(double), hipMemcpyDeviceToHost));
    return h;
  };
  const auto OBh4 = rd(sh.bOBh4, size_t(2) * NTG * nb * 3), OB3 = rd(sh.bOB3, size_t(2) * NTG * nb * 3);
  const auto Z5 = rd(sh.bZ5, size_t(2) * NTG * nb * 3), OB6 = rd(sh.bOB6, size_t(2) * NTG * nb);
  const auto W4 = rd(sh.bW4, size_t(2) * NTG * npm), X6 = rd(sh.bX6, size_t(2) * NTG * npm);
  const auto Wa = rd(sh.bWa, size_t(2) * NTG * npm);
  auto z = [](const std::vector<double>& v, size_t i) { return zc(v[2 * i], v[2 * i + 1]); };
  auto C = [&](int j, int g) { return zc(cb[2 * (size_t(j) * npm + g)], cb[2 * (size_t(j) * npm + g) + 1]); };
  // mesh side: per-spin n~(0) and const1 of the 3a2 correction (as in the corrections of the mesh targets)
  const int P = pb.P(), pnpm = pb.npw_max;
  std::vector<double> cm(size_t(2) * P * pnpm);
  TC_HIP(hipMemcpy(cm.data(), sh.coef.p, cm.size() * sizeof(double), hipMemcpyDeviceToHost));
  auto Cm = [&](int j, int g) { return zc(cm[2 * (size_t(j) * pnpm + g)], cm[2 * (size_t(j) * pnpm + g) + 1]); };
  double n0 = 0, cs = 0;
  for (int k = 0; k < pb.nk; ++k) {
    std::vector<zc> S(size_t(pb.nb) * pb.nb);
    for (int a = 0; a < pb.nb; ++a)
      for (int b = 0; b < pb.nb; ++b) {
        zc sacc = 0;
        for (int g = 0; g < pb.npw[k]; ++g) sacc += std::conj(Cm(k * pb.nb + a, g)) * Cm(k * pb.nb + b, g);
        S[size_t(a) * pb.nb + b] = sacc;
      }
    for (int a = 0; a < pb.nb; ++a) {
      const double fa = pb.occ[size_t(k) * pb.nb + a];
      n0 += fa / pb.nk * S[size_t(a) * pb.nb + a].real() / Om;
      for (int b = 0; b < pb.nb; ++b)
        cs += fa / pb.nk * pb.occ[size_t(k) * pb.nb + b] * (S[size_t(a) * pb.nb + b] * S[size_t(b) * pb.nb + a]).real() /
              (Om * Om);
    }
  }
  double c1a = 0, c1b_unit = 0;
  for (int ch = 0; ch < 2; ++ch) {
    const double A = pb.A[ch], Cc = pb.C[ch];
    const double nu = pb.reading == TC_DIV_LIMIT ? 2.0 : 1.0;   // u~_short(0)/N_k count of Eq. divcor_3a2_first
    c1a += kFourPi * A * (kFourPi * A * pb.delta_gb - nu * kFourPi * A * Cc * Cc / pb.nk);
    c1b_unit += 2.0 * kPi * A * kFourPi * A;   // times Delta_GB^band (Eq. 3b6_div_band1)
  }
  const double const1 = c1a * cs;
  for (int j = 0; j < NTG; ++j) {
    const int b = j / nb, q0 = b * nb;
    const double* V = &Vb[3 * b];
    const double VV = V[0] * V[0] + V[1] * V[1] + V[2] * V[2];
    auto f = [&](int mu) { return pb.bocc[size_t(b) * nb + mu]; };
    auto rho = [&](int mu, int jj) { return Sb[size_t(jj) * nb + mu] / Om; };   // <c_mu|c_jj> / Omega
    // per-mu coefficients of c_mu(G) and of (V . (k+G)) c_mu(G)
    std::vector<zc> al(nb, 0.0), be(nb, 0.0), ga(nb, 0.0), de(nb, 0.0);
    for (int mu = 0; mu < nb; ++mu) {
      const int qm = q0 + mu;
      const zc r = rho(mu, j);
      al[mu] += m.m2ax * (-kFourPi * dgbb[b]) * f(mu) * r;
      be[mu] += m.m2bx1 * (-a4) * f(mu) * r;
      zc X[3] = {0, 0, 0};
      for (int g = 0; g < pb.bnpw[b]; ++g) {
        const int* mi = &pb.bmiller[b][3 * g];
        const zc w = std::conj(C(qm, g)) * C(j, g);
        for (int cc = 0; cc < 3; ++cc)
          X[cc] += w * ((pb.bk[3 * b] + mi[0]) * pb.B[cc] + (pb.bk[3 * b + 1] + mi[1]) * pb.B[3 + cc] +
                        (pb.bk[3 * b + 2] + mi[2]) * pb.B[6 + cc]);
      }
      zc VX = 0, Vh4 = 0, V3 = 0, V5 = 0;
      for (int cc = 0; cc < 3; ++cc) {
        VX += V[cc] * X[cc] * zc(0, 1) / Om;
        Vh4 += V[cc] * z(OBh4, (size_t(j) * nb + mu) * 3 + cc) / Om;
        V3 += V[cc] * z(OB3, (size_t(j) * nb + mu) * 3 + cc) / Om;
        V5 += V[cc] * z(Z5, (size_t(j) * nb + mu) * 3 + cc) / Om;
      }
      al[mu] += m.m2bx2 * zc(0, -a4) * f(mu) * VX;
      al[mu] += 2.0 * m.m3b4 * zc(0, -0.5 * a4) * f(mu) * Vh4;
      al[mu] += 2.0 * m.m3b3 * zc(0, 0.5 * a4) * f(mu) * V3;
      ga[mu] += 2.0 * m.m3a4 * zc(0, 0.5 * a4) * f(mu) * r;                   // times (V . H3_mu)(G)
      al[mu] += 2.0 * m.m3b5 * zc(0, -0.5 * a4) * f(mu) * V5;
      de[mu] += 2.0 * m.m3b6 * f(mu) * r;                                      // times (F psi_mu)(G)
      al[mu] += 2.0 * m.m3b6 * f(mu) * (c1b_unit * dgbb[b] * n0 * r - z(OB6, size_t(j) * nb + mu) / Om);
      for (int m2 = 0; m2 < nb; ++m2) {
        // 3a4: mu plays mu1; 3b5: mu plays mu2 (partner index m2 plays mu1)
        al[mu] += 2.0 * m.m3a4 * 0.5 * a4 * a4 * VV * f(mu) * f(m2) * rho(mu, q0 + m2) * rho(m2, j);
        al[mu] += 2.0 * m.m3b5 * 0.5 * a4 * a4 * VV * f(mu) * f(m2) * rho(mu, q0 + m2) * rho(m2, j);
      }
    }
    for (int g = 0; g < pb.bnpw[b]; ++g) {
      const int* mi = &pb.bmiller[b][3 * g];
      double vk = 0;
      for (int cc = 0; cc < 3; ++cc)
        vk += V[cc] * ((pb.bk[3 * b] + mi[0]) * pb.B[cc] + (pb.bk[3 * b + 1] + mi[1]) * pb.B[3 + cc] +
                       (pb.bk[3 * b + 2] + mi[2]) * pb.B[6 + cc]);
      zc acc = m.m3a2 * 0.5 * (const1 * C(j, g) + z(Wa, size_t(j) * npm + g));
      for (int mu = 0; mu < nb; ++mu) {
        const int qm = q0 + mu;
        acc += (al[mu] + be[mu] * vk) * C(qm, g) + ga[mu] * z(W4, size_t(qm) * npm + g) +
               de[mu] * z(X6, size_t(qm) * npm + g);
      }
      out[2 * (size_t(j) * npm + g)] += acc.real();
      out[2 * (size_t(j) * npm + g) + 1] += acc.imag();
    }
  }
}

// The operator of the loaded (mesh) orbitals applied to the orbitals of the band k-points, and their
// orbital energies.
int do_apply_band(tc_ctx* c, double* out_host, double* eps_host) {
  Problem& pb = c->pb;
  Shared& sh = c->sh;
  if (pb.nkb == 0) return fail(c, TC_ERR_STATE, "no band k-points set");
  int st = prepare(c);
  if (st != TC_OK) return st;
  if (pb.bitc || pb.nspin == 2 || pb.nsym > 0)
    return fail(c, TC_ERR_UNSUPPORTED, "band k-points are built for TC mode with one spin channel and no symmetry");
  for (int b = 0; b < pb.nkb; ++b)
    if (!pb.bloaded[b]) return fail(c, TC_ERR_STATE, "orbitals of band k-point " + std::to_string(b) + " not loaded");
  const bool corr = pb.div && (pb.mask & TC_T_CORR);
  const int nkb = pb.nkb, nb = pb.bnb, npm = sh.bnpm;
  const int NTG = nkb * nb;
  // band GB quantities and the band orbitals' overlaps (FP64, host)
  if (corr && pb.band_alpha != pb.alpha) {   // the GB sums depend on the cell, mesh, alpha and band k-points
    pb.bdgb.assign(nkb, 0.0);
    pb.bVg.assign(size_t(3) * nkb, 0.0);
    for (int b = 0; b < nkb; ++b)
      if (!gb_band(pb, &pb.bk[3 * b], pb.bdgb[b], &pb.bVg[3 * b]))
        return fail(c, TC_ERR_ARG, "band k-point " + std::to_string(b) + " lies on the mesh: use the mesh k-point");
    pb.band_alpha = pb.alpha;
  }
  const std::vector<double> dgbb = corr ? pb.bdgb : std::vector<double>(nkb, 0.0);
  const std::vector<double> Vb = corr ? pb.bVg : std::vector<double>(size_t(3) * nkb, 0.0);
  std::vector<double> cb(size_t(2) * NTG * npm);
  TC_HIP(hipMemcpy(cb.data(), sh.bcoef.p, cb.size() * sizeof(double), hipMemcpyDeviceToHost));
  const double a4 = kFourPi * pb.A[0];   // 4 pi A of the parallel channel (exchange-type terms)
  using zc = std::complex<double>;
  auto coef = [&](int j, int g) { return zc(cb[2 * (size_t(j) * npm + g)], cb[2 * (size_t(j) * npm + g) + 1]); };
  std::vector<zc> Sb(size_t(NTG) * nb);   // Sb[j][mu] = <c_mu|c_j> (mu, j at the same band k-point)
  for (int j = 0; j < NTG; ++j)
    for (int mu = 0; mu < nb; ++mu) {
      const int b = j / nb, q = b * nb + mu;
      zc sacc = 0;
      for (int g = 0; g < pb.bnpw[b]; ++g) sacc += std::conj(coef(q, g)) * coef(j, g);
      Sb[size_t(j) * nb + mu] = sacc;
    }
  // plane-wave data of the band k-points
  std::vector<int> box(size_t(nkb) * npm, 0), tk(nkb);
  std::vector<double> kg(size_t(nkb) * npm * 3, 0.0);
  for (int b = 0; b < nkb; ++b) {
    tk[b] = pb.nk + b;
    for (int g = 0; g < pb.bnpw[b]; ++g) {
      const int* m = &pb.bmiller[b][3 * g];
      const int x = (m[0] % pb.N + pb.N) % pb.N, y = (m[1] % pb.N + pb.N) % pb.N, z = (m[2] % pb.N + pb.N) % pb.N;
      box[size_t(b) * npm + g] = (z * pb.N + y) * pb.N + x;
      for (int cc = 0; cc < 3; ++cc)
        kg[(size_t(b) * npm + g) * 3 + cc] = (pb.bk[3 * b] + m[0]) * pb.B[cc] + (pb.bk[3 * b + 1] + m[1]) * pb.B[3 + cc] +
                                             (pb.bk[3 * b + 2] + m[2]) * pb.B[6 + cc];
    }
  }
  sh.bbox.alloc(box.size());
  sh.bkg.alloc(kg.size());
  sh.bnpwd.alloc(nkb);
  sh.btk.alloc(nkb);
  sh.bout.alloc(size_t(2) * nkb * nb * npm);
  sh.beps.alloc(size_t(2) * nkb * nb);
  TC_HIP(hipMemcpy(sh.bbox.p, box.data(), box.size() * sizeof(int), hipMemcpyHostToDevice));
  TC_HIP(hipMemcpy(sh.bkg.p, kg.data(), kg.size() * sizeof(double), hipMemcpyHostToDevice));
  TC_HIP(hipMemcpy(sh.bnpwd.p, pb.bnpw.data(), nkb * sizeof(int), hipMemcpyHostToDevice));
  TC_HIP(hipMemcpy(sh.btk.p, tk.data(), nkb * sizeof(int), hipMemcpyHostToDevice));
  alloc_shared(c);
  TargetSet ts;
  ts.coef = sh.bcoef.p;
  ts.nvec = nb;
  ts.out = sh.bout.p;
  ts.nblk = nkb;
  ts.tk = sh.btk.p;
  ts.boxidx = sh.bbox.p;
  ts.npw = sh.bnpwd.p;
  ts.kg = sh.bkg.p;
  ts.npm = npm;
  ts.band = true;
  const Masks m = make_masks(pb.mask);
  if (corr) {
    // h4 correction coefficients a[j][mu] = -i 4 pi A f_mu S_mu,j / Omega (Eqs. divcorr_3a3, div_corr_3b4_2)
    std::vector<double> ah(size_t(2) * NTG * nb);
    for (int j = 0; j < NTG; ++j)
      for (int mu = 0; mu < nb; ++mu) {
        const zc v = zc(0, -a4) * pb.bocc[size_t(j / nb) * nb + mu] * Sb[size_t(j) * nb + mu] / pb.omega;
        ah[2 * (size_t(j) * nb + mu)] = v.real();
        ah[2 * (size_t(j) * nb + mu) + 1] = v.imag();
      }
    sh.bdh4.alloc(ah.size());
    sh.bV.alloc(Vb.size());
    TC_HIP(hipMemcpy(sh.bdh4.p, ah.data(), ah.size() * sizeof(double), hipMemcpyHostToDevice));
    TC_HIP(hipMemcpy(sh.bV.p, Vb.data(), Vb.size() * sizeof(double), hipMemcpyHostToDevice));
    for (auto* x : {&sh.bOBh4, &sh.bOB3, &sh.bZ5}) x->alloc(size_t(2) * NTG * nb * 3);
    sh.bOB6.alloc(size_t(2) * NTG * nb);
    for (auto* x : {&sh.bW4, &sh.bX6, &sh.bWa}) x->alloc(size_t(2) * NTG * npm);
    ts.bdh4 = sh.bdh4.p;
    ts.bV = sh.bV.p;
    ts.OBh4 = sh.bOBh4.p;
    ts.OB3 = sh.bOB3.p;
    ts.Z5 = sh.bZ5.p;
    ts.OB6 = sh.bOB6.p;
    ts.W4 = sh.bW4.p;
    ts.X6 = sh.bX6.p;
    ts.Wa = sh.bWa.p;
    ts.c3b6[0] = -2.0 * kPi * pb.A[0];
    ts.c3b6[1] = -2.0 * kPi * pb.A[1];
  }
  double stage[6];
  c->eng->prof = t_arena ? nullptr : &c->prof;
  c->eng->apply(c->stream, sh, pb, stage, &ts);
  std::vector<double> out(size_t(2) * NTG * npm);
  TC_HIP(hipMemcpyAsync(out.data(), sh.bout.p, out.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  TC_HIP(hipStreamSynchronize(c->stream));
  if (corr) band_corrections_host(c, m, cb, Sb, dgbb, Vb, out);
  // orbital energies <phi| T + h |phi> (FP64, host)
  std::vector<double> eps(size_t(2) * NTG);
  for (int j = 0; j < NTG; ++j) {
    const int b = j / nb;
    zc e = 0;
    for (int g = 0; g < pb.bnpw[b]; ++g) {
      const int* mi = &pb.bmiller[b][3 * g];
      double kg2 = 0;
      for (int cc = 0; cc < 3; ++cc) {
        const double q = (pb.bk[3 * b] + mi[0]) * pb.B[cc] + (pb.bk[3 * b + 1] + mi[1]) * pb.B[3 + cc] +
                         (pb.bk[3 * b + 2] + mi[2]) * pb.B[6 + cc];
        kg2 += q * q;
      }
      const zc cj = coef(j, g), hc(out[2 * (size_t(j) * npm + g)], out[2 * (size_t(j) * npm + g) + 1]);
      e += std::conj(cj) * (0.5 * kg2 * cj + hc);
    }
    eps[2 * j] = e.real();
    eps[2 * j + 1] = e.imag();
  }
  if (out_host) std::memcpy(out_host, out.data(), out.size() * sizeof(double));
  if (eps_host) std::memcpy(eps_host, eps.data(), eps.size() * sizeof(double));
  return TC_OK;
}

// ------------------------------------------------------------------ crystal symmetry (host)
// Integer inverse of a unimodular 3x3 matrix (row-major).
void int_inverse3(const int* R, int* Ri) {
  const int det = R[0] * (R[4] * R[8] - R[5] * R[7]) - R[1] * (R[3] * R[8] - R[5] * R[6]) +
                  R[2] * (R[3] * R[7] - R[4] * R[6]);
  const int adj[9] = {R[4] * R[8] - R[5] * R[7], R[2] * R[7] - R[1] * R[8], R[1] * R[5] - R[2] * R[4],
                      R[5] * R[6] - R[3] * R[8], R[0] * R[8] - R[2] * R[6], R[2] * R[3] - R[0] * R[5],
                      R[3] * R[7] - R[4] * R[6], R[1] * R[6] - R[0] * R[7], R[0] * R[4] - R[1] * R[3]};
  for (int i = 0; i < 9; ++i) Ri[i] = adj[i] / det;
}

// The image under operation o of mesh k-point k: index of R^T k (mod 1) and b = R^T k - k'
// (fractional units); false when R^T k is off the mesh.
bool sym_map_k(const Problem& pb, const int* R, int k, int* kout, int* b) {
  double f[3], g[3];
  pb.kfrac(k, f);
  const int n[3] = {pb.n1, pb.n2, pb.n3};
  int idx[3];
  for (int i = 0; i < 3; ++i) {
    g[i] = R[i] * f[0] + R[3 + i] * f[1] + R[6 + i] * f[2];   // (R^T f)_i
    const double x = g[i] * n[i] - pb.kshift[i];                 // mesh index of the image (shifted mesh)
    const double xr = std::round(x);
    if (std::fabs(x - xr) > 1e-9) return false;
    const int t = int(xr);
    idx[i] = ((t % n[i]) + n[i]) % n[i];
    b[i] = (t - idx[i]) / n[i];
  }
  *kout = (idx[0] * pb.n2 + idx[1]) * pb.n3 + idx[2];
  return true;
}

int set_symmetry(tc_ctx* c, int nsym, const int32_t* rot, const double* tau) {
  Problem& pb = c->pb;
  if (!pb.cell || pb.nk == 0 || pb.N == 0) return fail(c, TC_ERR_STATE, "set the cell, k-mesh and grid first");
  if (nsym < 0) return fail(c, TC_ERR_ARG, "nsym must be >= 0");
  pb.nsym = 0;
  pb.sym_ready = false;
  c->have_result = false;
  if (nsym == 0) return TC_OK;
  if (!rot || !tau) return fail(c, TC_ERR_ARG, "null operations");
  // lattice L (rows a_i) and its inverse
  const double* L = pb.lat;
  double Li[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Li[3 * i + j] = pb.B[3 * j + i] / (2 * kPi);   // L^-1 = B^T / 2 pi
  for (int o = 0; o < nsym; ++o) {
    const int* R = rot + 9 * o;
    const int det = R[0] * (R[4] * R[8] - R[5] * R[7]) - R[1] * (R[3] * R[8] - R[5] * R[6]) +
                    R[2] * (R[3] * R[7] - R[4] * R[6]);
    if (det != 1 && det != -1) return fail(c, TC_ERR_ARG, "operation " + std::to_string(o) + ": det R must be +-1");
    // S = L^T R L^-T must be orthogonal
    double S[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double v = 0;
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) v += L[3 * a + i] * R[3 * a + b] * Li[3 * j + b];
        S[3 * i + j] = v;
      }
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double v = 0;
        for (int a = 0; a < 3; ++a) v += S[3 * i + a] * S[3 * j + a];
        if (std::fabs(v - (i == j ? 1.0 : 0.0)) > 1e-9)
          return fail(c, TC_ERR_ARG, "operation " + std::to_string(o) + " is not an isometry of the lattice");
      }
    for (int i = 0; i < 3; ++i) {
      const double x = tau[3 * o + i] * pb.N;
      if (std::fabs(x - std::round(x)) > 1e-9)
        return fail(c, TC_ERR_ARG, "operation " + std::to_string(o) + ": N tau must be integer (grid-preserving)");
    }
    for (int k = 0; k < pb.nk; ++k) {
      int kk, b[3];
      if (!sym_map_k(pb, R, k, &kk, b))
        return fail(c, TC_ERR_ARG, "operation " + std::to_string(o) + " does not map the k-mesh onto itself");
    }
  }
  // closure: {R1|tau1}{R2|tau2} = x -> R1 R2 x + R1 R2 tau2 + R1 tau1 must be in the set (mod lattice)
  auto wvec = [&](const int* R, const double* t, double* w) {
    for (int i = 0; i < 3; ++i) w[i] = R[3 * i] * t[0] + R[3 * i + 1] * t[1] + R[3 * i + 2] * t[2];
  };
  auto same_mod1 = [](const double* a, const double* b) {
    for (int i = 0; i < 3; ++i) {
      const double d = a[i] - b[i];
      if (std::fabs(d - std::round(d)) > 1e-9) return false;
    }
    return true;
  };
  for (int o1 = 0; o1 < nsym; ++o1)
    for (int o2 = 0; o2 < nsym; ++o2) {
      const int *R1 = rot + 9 * o1, *R2 = rot + 9 * o2;
      int A[9];
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) A[3 * i + j] = R1[3 * i] * R2[j] + R1[3 * i + 1] * R2[3 + j] + R1[3 * i + 2] * R2[6 + j];
      double w2[3], w[3], w1[3];
      wvec(A, tau + 3 * o2, w2);
      wvec(R1, tau + 3 * o1, w1);
      for (int i = 0; i < 3; ++i) w[i] = w2[i] + w1[i];
      bool found = false;
      for (int o = 0; o < nsym && !found; ++o) {
        if (!std::equal(A, A + 9, rot + 9 * o)) continue;
        double wo[3];
        wvec(rot + 9 * o, tau + 3 * o, wo);
        found = same_mod1(w, wo);
      }
      if (!found) return fail(c, TC_ERR_ARG, "the operations do not form a group");
    }
  pb.symR.assign(rot, rot + 9 * nsym);
  pb.symT.assign(tau, tau + 3 * nsym);
  // orbits: the representative is the lowest k index of its orbit
  pb.krep.assign(pb.nk, -1);
  pb.kop.assign(pb.nk, -1);
  pb.kb.assign(3 * size_t(pb.nk), 0);
  pb.irr.clear();
  for (int k = 0; k < pb.nk; ++k) {
    if (pb.krep[k] >= 0) continue;
    pb.krep[k] = k;
    pb.irr.push_back(k);
    for (int o = 0; o < nsym; ++o) {
      int kk, b[3];
      sym_map_k(pb, rot + 9 * o, k, &kk, b);
      if (pb.krep[kk] >= 0) continue;
      pb.krep[kk] = k;
      pb.kop[kk] = o;
      for (int i = 0; i < 3; ++i) pb.kb[3 * kk + i] = b[i];
    }
  }
  pb.nsym = nsym;
  return TC_OK;
}

// Before the first application after a load: generates the orbitals (and fillings) of every
// non-representative k-point from its representative's, checks that each representative's weighted
// occupied set is invariant under its little group (the condition under which the fields of the images
// equal the directly computed ones), and uploads the expansion tables of sym.hpp.
int sym_prepare(tc_ctx* c) {
  Problem& pb = c->pb;
  Shared& sh = c->sh;
  const int nk = pb.nk, nb = pb.nb, npm = pb.npw_max, N = pb.N;
  const double* L = pb.lat;
  double Li[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Li[3 * i + j] = pb.B[3 * j + i] / (2 * kPi);
  std::vector<double> cf(size_t(2) * pb.P() * npm);
  TC_HIP(hipMemcpy(cf.data(), sh.coef.p, cf.size() * sizeof(double), hipMemcpyDeviceToHost));
  auto key = [](int a, int b, int d) { return ((long long)(a + 1024) << 22) | ((long long)(b + 1024) << 11) | (d + 1024); };
  // plane-wave lookup of each representative
  std::vector<std::unordered_map<long long, int>> look(nk);
  for (int r : pb.irr)
    for (int g = 0; g < pb.npw[r]; ++g) {
      const int* m = &pb.miller[r][3 * g];
      look[r][key(m[0], m[1], m[2])] = g;
    }
  // map of operation o with shift b from representative r onto a plane-wave list (miller, n):
  // g0[g] and the phase e^{2 pi i (m - b).tau}
  auto build_map = [&](int r, int o, const int* b, const std::vector<int>& mil, int n, int* g0, double* ph) -> bool {
    int Ri[9];
    int_inverse3(&pb.symR[9 * o], Ri);
    const double* t = &pb.symT[3 * o];
    for (int g = 0; g < n; ++g) {
      const int mb[3] = {mil[3 * g] - b[0], mil[3 * g + 1] - b[1], mil[3 * g + 2] - b[2]};
      int m0[3];
      for (int i = 0; i < 3; ++i) m0[i] = Ri[i] * mb[0] + Ri[3 + i] * mb[1] + Ri[6 + i] * mb[2];   // R^-T (m - b)
      auto it = look[r].find(key(m0[0], m0[1], m0[2]));
      if (it == look[r].end()) return false;
      g0[g] = it->second;
      const double phase = 2 * kPi * (mb[0] * t[0] + mb[1] * t[1] + mb[2] * t[2]);
      ph[2 * g] = std::cos(phase);
      ph[2 * g + 1] = std::sin(phase);
    }
    return true;
  };
  // little-group invariance of each representative's weighted occupied set
  for (int r : pb.irr) {
    const int n = pb.npw[r];
    std::vector<int> g0(n);
    std::vector<double> ph(2 * size_t(n));
    for (int o = 0; o < pb.nsym; ++o) {
      int kk, b[3];
      sym_map_k(pb, &pb.symR[9 * o], r, &kk, b);
      if (kk != r) continue;
      if (!build_map(r, o, b, pb.miller[r], n, g0.data(), ph.data()))
        return fail(c, TC_ERR_ARG, "plane waves of k-point " + std::to_string(r) + " are not invariant under its little group");
      // M[mu][nu] = <c_mu | O c_nu>; needs M M^H = 1 and M F = F M (F = fillings)
      std::vector<double> M(2 * size_t(nb) * nb, 0.0);
      for (int mu = 0; mu < nb; ++mu)
        for (int nu = 0; nu < nb; ++nu) {
          const double* x = &cf[2 * (size_t(r * nb + mu) * npm)];
          const double* y = &cf[2 * (size_t(r * nb + nu) * npm)];
          double sr = 0, si = 0;
          for (int g = 0; g < n; ++g) {
            const double yr = ph[2 * g] * y[2 * g0[g]] - ph[2 * g + 1] * y[2 * g0[g] + 1];
            const double yi = ph[2 * g] * y[2 * g0[g] + 1] + ph[2 * g + 1] * y[2 * g0[g]];
            sr += x[2 * g] * yr + x[2 * g + 1] * yi;
            si += x[2 * g] * yi - x[2 * g + 1] * yr;
          }
          M[2 * (mu * nb + nu)] = sr;
          M[2 * (mu * nb + nu) + 1] = si;
        }
      double err = 0;
      for (int i = 0; i < nb; ++i)
        for (int j = 0; j < nb; ++j) {
          double ur = 0, ui = 0;
          for (int l = 0; l < nb; ++l) {
            const double ar = M[2 * (i * nb + l)], ai = M[2 * (i * nb + l) + 1];
            const double br = M[2 * (j * nb + l)], bi = -M[2 * (j * nb + l) + 1];
            ur += ar * br - ai * bi;
            ui += ar * bi + ai * br;
          }
          err = std::max(err, std::hypot(ur - (i == j ? 1.0 : 0.0), ui));
          const double fi = pb.occ[size_t(r) * nb + i], fj = pb.occ[size_t(r) * nb + j];
          err = std::max(err, std::hypot(M[2 * (i * nb + j)], M[2 * (i * nb + j) + 1]) * std::fabs(fi - fj));
        }
      if (err > 1e-8)
        return fail(c, TC_ERR_ARG, "the occupied orbitals of k-point " + std::to_string(r) +
                                       " are not invariant under its little group (deviation " + std::to_string(err) + ")");
    }
  }
  // generation of the other k-points and the expansion tables
  std::vector<int> g0(size_t(nk) * npm, 0);
  std::vector<double> ph(size_t(2) * nk * npm, 0.0);
  std::vector<SymK> sk(nk);
  std::vector<int> rix(nk, -1);
  for (size_t i = 0; i < pb.irr.size(); ++i) rix[pb.irr[i]] = int(i);
  for (int k = 0; k < nk; ++k) {
    const int r = pb.krep[k], o = pb.kop[k];
    SymK& x = sk[k];
    x.rk = rix[r];
    if (o < 0) {
      for (int i = 0; i < 9; ++i) {
        x.R[i] = (i % 4 == 0);
        x.St[i] = (i % 4 == 0) ? 1.0 : 0.0;
      }
      for (int i = 0; i < 3; ++i) x.v[i] = x.b[i] = 0;
      for (int g = 0; g < pb.npw[k]; ++g) {
        g0[size_t(k) * npm + g] = g;
        ph[2 * (size_t(k) * npm + g)] = 1.0;
      }
      continue;
    }
    const int* R = &pb.symR[9 * o];
    const double* t = &pb.symT[3 * o];
    for (int i = 0; i < 9; ++i) x.R[i] = R[i];
    for (int i = 0; i < 3; ++i) {
      const double v = R[3 * i] * t[0] + R[3 * i + 1] * t[1] + R[3 * i + 2] * t[2];
      x.v[i] = int(std::lround(v * N));
      x.b[i] = pb.kb[3 * k + i];
    }
    // S^T = L^-1 R^T L (Cartesian)
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double v = 0;
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) v += Li[3 * i + a] * R[3 * b + a] * L[3 * b + j];
        x.St[3 * i + j] = v;
      }
    if (pb.npw[k] != pb.npw[r] ||
        !build_map(r, o, x.b, pb.miller[k], pb.npw[k], &g0[size_t(k) * npm], &ph[2 * size_t(k) * npm]))
      return fail(c, TC_ERR_ARG, "plane waves of k-point " + std::to_string(k) +
                                     " are not the image of those of k-point " + std::to_string(r));
    for (int mu = 0; mu < nb; ++mu) {
      double* dst = &cf[2 * (size_t(k * nb + mu) * npm)];
      const double* src = &cf[2 * (size_t(r * nb + mu) * npm)];
      for (int g = 0; g < npm; ++g) {
        double re = 0, im = 0;
        if (g < pb.npw[k]) {
          const int s0 = g0[size_t(k) * npm + g];
          const double pr = ph[2 * (size_t(k) * npm + g)], pi = ph[2 * (size_t(k) * npm + g) + 1];
          re = pr * src[2 * s0] - pi * src[2 * s0 + 1];
          im = pr * src[2 * s0 + 1] + pi * src[2 * s0];
        }
        dst[2 * g] = re;
        dst[2 * g + 1] = im;
      }
      pb.occ[size_t(k) * nb + mu] = pb.occ[size_t(r) * nb + mu];
    }
    pb.loaded[k] = 1;
  }
  TC_HIP(hipMemcpy(sh.coef.p, cf.data(), cf.size() * sizeof(double), hipMemcpyHostToDevice));
  upload_basis_data(c);
  sh.symk.alloc(nk);
  sh.irrk.alloc(pb.irr.size());
  sh.symg0.alloc(g0.size());
  sh.symph.alloc(ph.size());
  TC_HIP(hipMemcpy(sh.symk.p, sk.data(), sk.size() * sizeof(SymK), hipMemcpyHostToDevice));
  TC_HIP(hipMemcpy(sh.irrk.p, pb.irr.data(), pb.irr.size() * sizeof(int), hipMemcpyHostToDevice));
  TC_HIP(hipMemcpy(sh.symg0.p, g0.data(), g0.size() * sizeof(int), hipMemcpyHostToDevice));
  TC_HIP(hipMemcpy(sh.symph.p, ph.data(), ph.size() * sizeof(double), hipMemcpyHostToDevice));
  pb.sym_ready = true;
  return TC_OK;
}

int prepare(tc_ctx* c) {
  Problem& pb = c->pb;
  if (!pb.cell) return fail(c, TC_ERR_STATE, "tc_set_cell not called");
  if (pb.nk == 0) return fail(c, TC_ERR_STATE, "tc_set_kmesh not called");
  if (pb.N == 0) return fail(c, TC_ERR_STATE, "tc_set_grid not called");
  if (!pb.jastrow) return fail(c, TC_ERR_STATE, "tc_set_jastrow not called");
  if (pb.nb == 0) return fail(c, TC_ERR_STATE, "no orbitals loaded");
  int nleft = 0;
  for (int k = 0; k < pb.nk; ++k) {
    // with symmetry, the orbitals of k-points other than the representatives are generated
    if (!pb.loaded[k] && !(pb.nsym > 0 && pb.krep[k] != k))
      return fail(c, TC_ERR_STATE, "orbitals of k-point " + std::to_string(k) + " not loaded");
    nleft += pb.left[k];
  }
  if (pb.nspin == 2) {
    for (int k = 0; k < pb.nk; ++k) {
      if (!pb.loaded_dn[k])
        return fail(c, TC_ERR_STATE, "down-spin orbitals of k-point " + std::to_string(k) + " not loaded");
      nleft += pb.left_dn[k];
    }
  }
  if (pb.nsym > 0 && (nleft != 0 || pb.nspin == 2))
    return fail(c, TC_ERR_UNSUPPORTED, "symmetry is built for TC mode with one spin channel");
  if (nleft != 0 && nleft != pb.nspin * pb.nk)
    return fail(c, TC_ERR_STATE, "left orbitals are loaded for some k-points or spin channels only");
  pb.bitc = nleft != 0;
  if (!c->eng || c->eng_prec != pb.prec || c->eng_N != pb.N) {
    if (pb.prec == TC_PREC_FP32_SPLITBF16 && pb.N % 8 != 0)
      return fail(c, TC_ERR_UNSUPPORTED, "split-BF16 DFT stages need a grid length divisible by 8");
    c->eng.reset(pb.prec == TC_PREC_FP64 ? make_engine_r<double>(pb.N)
                                         : make_engine_r<float>(pb.N, pb.prec == TC_PREC_FP32_SPLITBF16));
    if (!c->eng) return fail(c, TC_ERR_UNSUPPORTED, "grid not supported");
    c->eng_prec = pb.prec;
    c->eng_N = pb.N;
    c->tables_dirty = true;
  }
  if (c->tables_dirty) {
    gb_constant(pb);
    c->eng->upload_tables(pb, TableVariant{});
    c->tables_dirty = false;
  }
  if (pb.nsym > 0 && !pb.sym_ready) return sym_prepare(c);
  return TC_OK;
}

void finish_energy(tc_ctx* c) {
  Problem& pb = c->pb;
  const int P = pb.P();
  const Masks m = make_masks(pb.mask);
  const int ns = pb.nspin;
  std::vector<double> ep(size_t(kAccSlots) * ns * P), tk(size_t(ns) * P), ec(size_t(2) * ns * P);
  TC_HIP(hipMemcpy(ep.data(), c->sh.epart.p, ep.size() * sizeof(double), hipMemcpyDeviceToHost));
  TC_HIP(hipMemcpy(tk.data(), c->sh.tkin.p, tk.size() * sizeof(double), hipMemcpyDeviceToHost));
  TC_HIP(hipMemcpy(ec.data(), c->sh.ecorr.p, ec.size() * sizeof(double), hipMemcpyDeviceToHost));
  double T = 0, E2 = 0, E3 = 0, EC = 0;
  for (int p = 0; p < ns * P; ++p) {
    // unpolarised: both spin channels (factor 2); polarised: each channel with its own fillings
    const double f = ns == 1 ? pb.occ[p] * 2.0 / pb.nk : (p < P ? pb.occ[p] : pb.occ_dn[p - P]) / pb.nk;
    const double* e = &ep[size_t(kAccSlots) * p];
    T += f * tk[p];
    // Two-body terms count 1/2, three-body terms 1/3 (multiplicities are in the operator).  Pass B (slot 3)
    // fuses 2bx2 with 3b3-3b5 (and 3b6); the 2bx2 bracket equals the 2bx1 bracket (slot 1, accumulated whenever
    // either is selected) because the discrete kernels are transposes of each other, so it is moved from
    // the 1/3 to the 1/2 group through slot 1.
    E2 += f * 0.5 * (e[0] + e[4] + e[5] + (m.m2bx1 + m.m2bx2) * e[1]);
    E3 += f * (e[2] + e[3] - m.m2bx2 * e[1]) / 3.0;
    E2 += f * 0.5 * ec[2 * p];
    E3 += f * ec[2 * p + 1] / 3.0;
    EC += f * (0.5 * ec[2 * p] + ec[2 * p + 1] / 3.0);
  }
  c->e_parts[TC_E_KINETIC] = T;
  c->e_parts[TC_E_TWO_BODY] = E2;
  c->e_parts[TC_E_THREE_BODY] = E3;
  c->e_parts[TC_E_CORR] = EC;
  c->e_total = T + E2 + E3;
}

// One application with whatever tables are uploaded; energies kept for tc_energy.
void alloc_shared(tc_ctx* c) {
  Problem& pb = c->pb;
  Shared& sh = c->sh;
  const int P = pb.nspin * pb.P();   // orbitals of all spin channels
  sh.out.alloc(size_t(2) * P * pb.npw_max);
  sh.dhc2.alloc(size_t(2) * P * pb.npw_max);
  sh.dhc3.alloc(size_t(2) * P * pb.npw_max);
  sh.Zg.alloc(size_t(2) * P * pb.npw_max);
  sh.Wg.alloc(size_t(2) * P * pb.npw_max);
  sh.epart.alloc(size_t(kAccSlots) * P);
  sh.tkin.alloc(P);
  sh.ecorr.alloc(size_t(2) * P);
  sh.S.alloc(size_t(2) * pb.nk * pb.nb * pb.nb);
  sh.O.alloc(size_t(2) * pb.nk * pb.nb * pb.nb);
  sh.eps.alloc(size_t(2) * P);
}

void run_apply(tc_ctx* c, void* out_dev, double* out_host) {
  Problem& pb = c->pb;
  Shared& sh = c->sh;
  const int P = pb.nspin * pb.P();   // orbitals of all spin channels (spin-major)
  alloc_shared(c);
  c->eng->prof = t_arena ? nullptr : &c->prof;
  c->eng->apply(c->stream, sh, pb, c->stage_ms);
  c->total_ms = 0;
  for (double v : c->stage_ms) c->total_ms += v;
  for (int sp = 0; sp < pb.nspin; ++sp) {
    const size_t co = size_t(2) * sp * pb.P() * pb.npw_max;
    hipLaunchKernelGGL(k_orbital_eps, dim3(pb.P()), dim3(256), 0, c->stream, (pb.bitc ? sh.coefL.p : sh.coef.p) + co,
                       sh.coef.p + co, sh.out.p + co, sh.kg.p, sh.npw.p, pb.nb, pb.npw_max,
                       sh.eps.p + size_t(2) * sp * pb.P());
  }
  c->eps.resize(size_t(2) * P);
  TC_HIP(hipMemcpyAsync(c->eps.data(), sh.eps.p, c->eps.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  if (out_dev)
    TC_HIP(hipMemcpyAsync(out_dev, sh.out.p, size_t(2) * P * pb.npw_max * sizeof(double), hipMemcpyDeviceToDevice,
                          c->stream));
  if (out_host)
    TC_HIP(hipMemcpyAsync(out_host, sh.out.p, size_t(2) * P * pb.npw_max * sizeof(double), hipMemcpyDeviceToHost,
                          c->stream));
  TC_HIP(hipStreamSynchronize(c->stream));
  finish_energy(c);
  c->have_result = true;
}

int do_apply(tc_ctx* c, void* out_dev, double* out_host) {
  int st = prepare(c);
  if (st != TC_OK) return st;
  run_apply(c, out_dev, out_host);
  return TC_OK;
}

// tc_apply_all_dev with every device buffer of the call carved from the scratch.  The context must have
// been prepared by an ordinary application since its last change (kernel tables and engine exist), so
// that nothing outside the call's own buffers is made.
int do_apply_noalloc(tc_ctx* c, void* out_dev) {
  Problem& pb = c->pb;
  if (!out_dev) return fail(c, TC_ERR_ARG, "out_dev must not be NULL");
  if (!c->eng || c->tables_dirty || c->eng_prec != pb.prec || c->eng_N != pb.N || (pb.nsym > 0 && !pb.sym_ready))
    return fail(c, TC_ERR_STATE,
                "the context is not prepared: run tc_apply_all_dev (or tc_apply_all) once after the last change");
  const int st = prepare(c);
  if (st != TC_OK) return st;
  if (!c->scratch) return fail(c, TC_ERR_DEVICE, "no scratch on this device");
  TC_HIP(hipStreamSynchronize(c->stream));   // the scratch is free: the previous call on this stream is done
  ArenaScope scope(c->scratch);
  run_apply(c, out_dev, nullptr);
  return TC_OK;
}

// The operator of the loaded orbitals applied to nvec trial vectors per k-point (device in/out).
int do_apply_vectors(tc_ctx* c, int nvec, const double* in_dev, double* out_dev) {
  if (nvec <= 0) return fail(c, TC_ERR_ARG, "nvec must be positive");
  if (c->pb.nsym > 0) return fail(c, TC_ERR_UNSUPPORTED, "trial vectors are built without symmetry");
  int st = prepare(c);
  if (st != TC_OK) return st;
  alloc_shared(c);
  TargetSet ts;
  ts.coef = in_dev;
  ts.nvec = nvec;
  ts.out = out_dev;
  double stage[6];
  c->eng->prof = t_arena ? nullptr : &c->prof;
  c->eng->apply(c->stream, c->sh, c->pb, stage, &ts);
  TC_HIP(hipStreamSynchronize(c->stream));
  return TC_OK;
}

constexpr uint64_t kTermsB = TC_T_2BH1 | TC_T_2BH2 | TC_T_2BX1 | TC_T_2BX2;
constexpr uint64_t kTerms3 = TC_T_3A1 | TC_T_3A2 | TC_T_3A3 | TC_T_3A4 | TC_T_3B1 | TC_T_3B2 | TC_T_3B3 | TC_T_3B4 |
                             TC_T_3B5 | TC_T_3B6;

// Gradient of the energy of the loaded orbitals.
//  * Orbitals: the two-body V2a terms (with C2ax) and the whole three-body operator (with its
//    corrections) are the exact first variations of their energies and are Hermitian in the discrete
//    form, so their gradient is 4 w_p h c_p.  The grad-u . grad terms are not Hermitian: their
//    gradient is minus the pair operator with kernel L~ = -Q^2 u~ (zero at Q = 0).  Both are obtained
//    by one application with V2a replaced by V2a - L~ and the grad-u . grad terms off.
//  * A and C: central differences along exact tangent tables (TableVariant::TANGENT), exact because
//    the energy is quadratic in the tables and correction prefactors taken together.
int do_backward(tc_ctx* c, void* grad_dev, double* grad_host, double* dA, double* dC, void* gl_dev = nullptr,
                double* gl_host = nullptr) {
  Problem& pb = c->pb;
  const uint64_t m = pb.mask;
  if ((m & kTermsB) != 0 && (m & kTermsB) != kTermsB)
    return fail(c, TC_ERR_UNSUPPORTED, "the gradient needs 2bh1, 2bh2, 2bx1 and 2bx2 selected together");
  if ((m & kTerms3) != 0 && (m & kTerms3) != kTerms3)
    return fail(c, TC_ERR_UNSUPPORTED, "the gradient needs all three-body terms or none");
  if ((m & kTermsB) != 0 && (m & (TC_T_2AH | TC_T_2AX)) != (TC_T_2AH | TC_T_2AX))
    return fail(c, TC_ERR_UNSUPPORTED, "the gradient of the grad-u . grad terms needs 2ah and 2ax selected");
  int st = prepare(c);
  if (st != TC_OK) return st;
  if (pb.nsym > 0) return fail(c, TC_ERR_UNSUPPORTED, "the gradient is built without symmetry");
  if (!pb.bitc && (gl_dev || gl_host)) return fail(c, TC_ERR_ARG, "no left orbitals loaded: grad_left must be NULL");
  struct Keep {
    tc_ctx* c;
    uint64_t mask;
    double e, parts[TC_E_NPARTS], stage[6], total;
    bool had;
    std::vector<double> eps;
    bool swapped = false;
    ~Keep() {
      if (swapped) {
        std::swap(c->sh.coef.p, c->sh.coefL.p);
        std::swap(c->sh.coef.n, c->sh.coefL.n);
      }
      c->pb.negate_b = false;
      c->pb.force_rem = false;
      c->pb.mask = mask;
      c->tables_dirty = true;   // the next application rebuilds the operator's tables
      c->e_total = e;
      std::memcpy(c->e_parts, parts, sizeof(parts));
      std::memcpy(c->stage_ms, stage, sizeof(stage));
      c->total_ms = total;
      c->have_result = had;
      c->eps = eps;
    }
  } keep{c, m, c->e_total, {}, {}, c->total_ms, c->have_result, c->eps};
  std::memcpy(keep.parts, c->e_parts, sizeof(keep.parts));
  std::memcpy(keep.stage, c->stage_ms, sizeof(keep.stage));
  Shared& sh = c->sh;
  const int P = pb.P();
  const size_t bytes = size_t(2) * P * pb.npw_max * sizeof(double);
  // per spin channel (spin-major, as the operator output): scale w_p (h c_p + |k+G|^2/2 c_p)
  auto finish = [&](double scale, void* ddev, double* dhost) {
    const size_t per = size_t(2) * P * pb.npw_max;   // doubles per channel
    sh.grad.alloc(per * pb.nspin);
    for (int sp = 0; sp < pb.nspin; ++sp)
      hipLaunchKernelGGL(k_grad_finish, dim3(nblk(long(P) * pb.npw_max)), dim3(256), 0, c->stream,
                         sh.coef.p + sp * per, sh.out.p + sp * per, sh.kg.p, sh.npw.p, sh.w.p + sp * P, pb.nb,
                         pb.npw_max, P, scale, sh.grad.p + sp * per);
    if (ddev) TC_HIP(hipMemcpyAsync(ddev, sh.grad.p, bytes * pb.nspin, hipMemcpyDeviceToDevice, c->stream));
    if (dhost) TC_HIP(hipMemcpyAsync(dhost, sh.grad.p, bytes * pb.nspin, hipMemcpyDeviceToHost, c->stream));
    TC_HIP(hipStreamSynchronize(c->stream));
  };
  if (!pb.bitc) {
    if (grad_dev || grad_host) {
      pb.mask = m & ~kTermsB;
      pb.force_rem = (m & TC_T_2BX1) != 0;   // the 2bx1 remainder is Hermitian: it stays in the gradient
      c->tables_dirty = true;
      c->eng->upload_tables(pb, TableVariant{TableVariant::GRADIENT, 0, 0.0});
      run_apply(c, nullptr, nullptr);
      // 2 dE/dc* = 2 w (T + h_grad) c per channel's own coefficients; unpolarised, both channels share
      // them and the two contributions add (factor 4)
      finish(pb.nspin == 2 ? 2.0 : 4.0, grad_dev, grad_host);
      pb.mask = m;
      pb.force_rem = false;
    }
  } else {
    // E = Re sum f <chi| T + h2/2 + h3/3 |phi> with the pair held fixed:
    //   2 dE/dchi* = 2 w (T + h) phi                    (Eq. BITCSCF: the operator itself)
    //   2 dE/dphi* = 2 w (T + h^dagger) chi             (Eq. BITCSCFconj: the left operator)
    // h^dagger is the operator with chi and phi exchanged and v2 replaced by its adjoint: the
    // grad-u . grad terms change sign and the scalar kernel becomes V2a - 2 L~ (the discrete adjoint of
    // those terms is minus themselves minus twice the pair operator with kernel L~; their sum with the
    // operator gives the V2a - L~ of the TC gradient).
    if (gl_dev || gl_host) {
      c->tables_dirty = true;
      c->eng->upload_tables(pb, TableVariant{});
      run_apply(c, nullptr, nullptr);
      // 2 dE/dchi* per channel: one spin channel per orbital set when polarised, both otherwise
      finish(pb.nspin == 2 ? 1.0 : 2.0, gl_dev, gl_host);
    }
    if (grad_dev || grad_host) {
      std::swap(sh.coef.p, sh.coefL.p);
      std::swap(sh.coef.n, sh.coefL.n);
      keep.swapped = true;
      pb.negate_b = true;
      c->tables_dirty = true;
      c->eng->upload_tables(pb, TableVariant{TableVariant::ADJOINT, 0, 0.0});
      run_apply(c, nullptr, nullptr);
      finish(pb.nspin == 2 ? 1.0 : 2.0, grad_dev, grad_host);
      std::swap(sh.coef.p, sh.coefL.p);
      std::swap(sh.coef.n, sh.coefL.n);
      keep.swapped = false;
      pb.negate_b = false;
    }
  }
  for (int dir = 0; dir < 4; ++dir) {
    double* dst = dir < 2 ? (dA ? dA + dir : nullptr) : (dC ? dC + dir - 2 : nullptr);
    if (!dst) continue;
    const double th = dir < 2 ? pb.A[dir] : pb.C[dir - 2];
    const double h = std::max(std::fabs(th), 0.1);
    double e[2];
    for (int sgn = 0; sgn < 2; ++sgn) {
      c->tables_dirty = true;
      c->eng->upload_tables(pb, TableVariant{TableVariant::TANGENT, dir, sgn ? -h : h});
      run_apply(c, nullptr, nullptr);
      e[sgn] = c->e_total;
    }
    *dst = (e[0] - e[1]) / (2.0 * h);
  }
  return TC_OK;
}

void upload_basis_data(tc_ctx* c) {
  Problem& pb = c->pb;
  const int P = pb.P();
  std::vector<int> box(size_t(pb.nk) * pb.npw_max, 0);
  std::vector<double> kg(size_t(pb.nk) * pb.npw_max * 3, 0.0);
  for (int k = 0; k < pb.nk; ++k) {
    double f[3];
    pb.kfrac(k, f);
    for (int g = 0; g < pb.npw[k]; ++g) {
      const int* m = &pb.miller[k][3 * g];
      const int x = (m[0] % pb.N + pb.N) % pb.N, y = (m[1] % pb.N + pb.N) % pb.N, z = (m[2] % pb.N + pb.N) % pb.N;
      box[size_t(k) * pb.npw_max + g] = (z * pb.N + y) * pb.N + x;
      for (int cc = 0; cc < 3; ++cc)
        kg[(size_t(k) * pb.npw_max + g) * 3 + cc] =
            (f[0] + m[0]) * pb.B[cc] + (f[1] + m[1]) * pb.B[3 + cc] + (f[2] + m[2]) * pb.B[6 + cc];
    }
  }
  c->sh.boxidx.alloc(box.size());
  c->sh.kg.alloc(kg.size());
  c->sh.npw.alloc(pb.nk);
  c->sh.w.alloc(size_t(pb.nspin) * P);
  std::vector<double> w(size_t(pb.nspin) * P);
  for (int p = 0; p < P; ++p) w[p] = pb.occ[p] / pb.nk;
  if (pb.nspin == 2)
    for (int p = 0; p < P; ++p) w[P + p] = pb.occ_dn[p] / pb.nk;
  TC_HIP(hipMemcpy(c->sh.boxidx.p, box.data(), box.size() * sizeof(int), hipMemcpyHostToDevice));
  TC_HIP(hipMemcpy(c->sh.kg.p, kg.data(), kg.size() * sizeof(double), hipMemcpyHostToDevice));
  TC_HIP(hipMemcpy(c->sh.npw.p, pb.npw.data(), pb.nk * sizeof(int), hipMemcpyHostToDevice));
  TC_HIP(hipMemcpy(c->sh.w.p, w.data(), w.size() * sizeof(double), hipMemcpyHostToDevice));
}

int begin_load(tc_ctx* c, int ik, int nband, const double* occ, int spin = 0) {
  Problem& pb = c->pb;
  if (pb.nk == 0 || pb.N == 0) return fail(c, TC_ERR_STATE, "set the k-mesh and grid before loading orbitals");
  if (ik < 0 || ik >= pb.nk) return fail(c, TC_ERR_ARG, "k-point index out of range");
  for (int k = 0; k < pb.nk; ++k)
    if (pb.npw[k] <= 0) return fail(c, TC_ERR_STATE, "tc_set_basis missing for k-point " + std::to_string(k));
  if (nband <= 0 || !occ) return fail(c, TC_ERR_ARG, "nband must be positive and occ non-null");
  if (nband > pb.npw[ik]) return fail(c, TC_ERR_ARG, "more bands than plane waves");
  for (int b = 0; b < nband; ++b)
    if (!(occ[b] >= 0.0 && occ[b] <= 1.0)) return fail(c, TC_ERR_ARG, "fillings must lie in [0, 1]");
  if (pb.nb != nband) {
    if (pb.nb != 0)
      for (int k = 0; k < pb.nk; ++k)
        if ((pb.loaded[k] && (k != ik || spin != 0)) || (pb.nspin == 2 && pb.loaded_dn[k] && (k != ik || spin != 1)))
          return fail(c, TC_ERR_ARG, "nband differs between k-points or spin channels");
    pb.nb = nband;
    pb.occ.assign(size_t(pb.nk) * nband, 0.0);
    pb.occ_dn.assign(size_t(pb.nk) * nband, 0.0);
    std::fill(pb.loaded.begin(), pb.loaded.end(), 0);
    std::fill(pb.left.begin(), pb.left.end(), 0);
    std::fill(pb.loaded_dn.begin(), pb.loaded_dn.end(), 0);
    std::fill(pb.left_dn.begin(), pb.left_dn.end(), 0);
  }
  int mx = 0;
  for (int k = 0; k < pb.nk; ++k) mx = std::max(mx, pb.npw[k]);
  pb.npw_max = mx;
  c->sh.coef.alloc(size_t(2) * pb.nspin * pb.P() * pb.npw_max);   // spin-major: spin 0 first
  double* o = spin == 0 ? pb.occ.data() : pb.occ_dn.data();
  for (int b = 0; b < nband; ++b) o[size_t(ik) * nband + b] = occ[b];
  pb.sym_ready = false;
  return TC_OK;
}

// FP64 biorthogonalisation of k-point ik on the device (see k_bo_normalize / k_bo_invert / k_bo_left):
// the right coefficients in sh.coef are normalised in place, the left ones (staged in sh.bo_l) are
// written to sh.coefL.
// Same for nb bands of k-point ik held elsewhere: right (normalised in place), the left set staged in
// sh.bo_l, the biorthogonalised left set written to lout.
int biorthogonalize_at(tc_ctx* c, int ik, int nb, double* right, double* lout) {
  Problem& pb = c->pb;
  Shared& sh = c->sh;
  const int npw = pb.npw[ik], npm = pb.npw_max;
  sh.bo_s.alloc(size_t(2) * nb * nb);
  sh.bo_inv.alloc(size_t(2) * nb * nb);
  sh.bo_aug.alloc(size_t(2) * (size_t(nb) * 2 * nb + nb));
  sh.bo_flag.alloc(1);
  hipStream_t s = c->stream;
  TC_HIP(hipMemsetAsync(sh.bo_flag.p, 0, sizeof(int), s));
  hipLaunchKernelGGL(k_bo_normalize, dim3(nb), dim3(256), 0, s, right, npw, npm, sh.bo_flag.p);
  hipLaunchKernelGGL(k_overlap, dim3(nb * nb), dim3(256), 0, s, sh.bo_l.p, nb, right, nb, sh.npw.p + ik, npm, 1,
                     sh.bo_s.p);
  hipLaunchKernelGGL(k_bo_invert, dim3(1), dim3(256), 0, s, sh.bo_s.p, nb, sh.bo_aug.p, sh.bo_inv.p, sh.bo_flag.p);
  int flag = 0;
  TC_HIP(hipMemcpyAsync(&flag, sh.bo_flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
  TC_HIP(hipStreamSynchronize(s));
  if (flag == 1) return fail(c, TC_ERR_ARG, "a right orbital of k-point " + std::to_string(ik) + " is zero");
  if (flag == 2)
    return fail(c, TC_ERR_ARG, "the left/right overlap of k-point " + std::to_string(ik) + " is singular");
  hipLaunchKernelGGL(k_bo_left, dim3(nblk(long(nb) * npm)), dim3(256), 0, s, sh.bo_inv.p, sh.bo_l.p, nb, npw, npm,
                     lout);
  TC_HIP(hipStreamSynchronize(s));
  return TC_OK;
}

int biorthogonalize(tc_ctx* c, int ik) {
  Problem& pb = c->pb;
  const size_t off = size_t(2) * ik * pb.nb * pb.npw_max;
  c->sh.coefL.alloc(size_t(2) * pb.nspin * pb.P() * pb.npw_max);   // spin-major, as the right coefficients
  return biorthogonalize_at(c, ik, pb.nb, c->sh.coef.p + off, c->sh.coefL.p + off);
}

// Replace the context's orbital set by nbx bands per k-point from device buffers ([nk][nbx][npw_max]
// complex128; left may be null) with fillings occ ([nk][nbx]).
// Load nbx orbitals per k-point (per channel and k-point with two spin channels: r and occ channel-major,
// the first nk nbx fillings for channel 0).
void load_set(tc_ctx* c, const double* r, const double* l, int nbx, const std::vector<double>& occ) {
  Problem& pb = c->pb;
  pb.nb = nbx;
  const size_t per = size_t(pb.nk) * nbx;
  pb.occ.assign(occ.begin(), occ.begin() + per);
  if (pb.nspin == 2) {
    pb.occ_dn.assign(occ.begin() + per, occ.begin() + 2 * per);
    std::fill(pb.loaded_dn.begin(), pb.loaded_dn.end(), 1);
    std::fill(pb.left_dn.begin(), pb.left_dn.end(), l ? 1 : 0);
  }
  std::fill(pb.loaded.begin(), pb.loaded.end(), 1);
  std::fill(pb.left.begin(), pb.left.end(), l ? 1 : 0);
  const size_t n = size_t(2) * pb.nspin * pb.P() * pb.npw_max;
  c->sh.coef.alloc(n);
  TC_HIP(hipMemcpyAsync(c->sh.coef.p, r, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  if (l) {
    c->sh.coefL.alloc(n);
    TC_HIP(hipMemcpyAsync(c->sh.coefL.p, l, n * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  }
  TC_HIP(hipStreamSynchronize(c->stream));
  upload_basis_data(c);
  c->have_result = false;
}

// Block-Davidson TC / BITC self-consistent loop (Sec. 2.4).  Each iteration: the current right orbitals,
// orthonormalised, start the subspace; pmax blocks of Payne-preconditioned residuals
// P (h - eps_i) v_{(p-1) nb + i} are added with Gram-Schmidt (dropping negligible or dependent vectors);
// the subspace matrix <v_a|T + h|v_b> is diagonalised and the nb eigenvectors of lowest real eigenvalue
// become the new orbitals (TC: Gram-Schmidt orthonormalised; BITC: right and left eigenvectors, then
// biorthonormalised), so the operator is updated every loop.  The loop ends when the energy changes by
// less than etol.
int do_scf(tc_ctx* c, const tc_scf_params& prm, double* ehist, int* niter) {
  if (prm.max_iter < 1 || prm.pmax < 0 || prm.pmax > 16 || !(prm.etol > 0) || !(prm.mix > 0 && prm.mix <= 1))
    return fail(c, TC_ERR_ARG,
                "scf parameters out of range (max_iter >= 1, 0 <= pmax <= 16, etol > 0, 0 < mix <= 1)");
  int st = prepare(c);
  if (st != TC_OK) return st;
  if (c->pb.nsym > 0) return fail(c, TC_ERR_UNSUPPORTED, "the self-consistent loop is built without symmetry");
  Problem& pb = c->pb;
  Shared& sh = c->sh;
  hipStream_t s = c->stream;
  const bool bitc = pb.bitc;
  // two spin channels (Eq. SCF per spin): each (channel, k-point) pair is one subspace block of its own
  // (nk below counts them), and one application serves the trial vectors of both channels
  const int ns = pb.nspin;
  const int nk = ns * pb.nk, nb = pb.nb, npm = pb.npw_max, P = ns * pb.P();
  const int nblk_sub = prm.pmax + 1, M = nblk_sub * nb;
  if (M > 512) return fail(c, TC_ERR_UNSUPPORTED, "subspace larger than 512 vectors per k-point");
  std::vector<double> f = pb.occ;              // fillings of the orbitals, [channel][nk][nb]
  if (ns == 2) f.insert(f.end(), pb.occ_dn.begin(), pb.occ_dn.end());
  const int* npwx = sh.npw.p;                  // plane-wave counts and k + G per block
  const double* kgx = sh.kg.p;
  if (ns == 2) {
    const int nk1 = pb.nk;
    c->dnpw2.alloc(2 * size_t(nk1));
    c->dkg2.alloc(size_t(2) * nk1 * npm * 3);
    for (int h = 0; h < 2; ++h) {
      TC_HIP(hipMemcpyAsync(c->dnpw2.p + h * nk1, sh.npw.p, nk1 * sizeof(int), hipMemcpyDeviceToDevice, s));
      TC_HIP(hipMemcpyAsync(c->dkg2.p + size_t(h) * nk1 * npm * 3, sh.kg.p, size_t(nk1) * npm * 3 * sizeof(double),
                            hipMemcpyDeviceToDevice, s));
    }
    npwx = c->dnpw2.p;
    kgx = c->dkg2.p;
  }
  const size_t blk = size_t(2) * P * npm;      // doubles per block of nb bands on every k-point
  const size_t kb = size_t(2) * nb * npm;      // doubles per k-point within a block
  c->dV.alloc(nblk_sub * blk);
  c->dHV.alloc(nblk_sub * blk);
  c->dHs.alloc(size_t(2) * nk * M * M);
  c->dwork.alloc(size_t(2) * nk * (4 * size_t(M) * M + 2 * M));
  c->dX.alloc(size_t(2) * nk * M * nb);
  c->dY.alloc(size_t(2) * nk * M * nb);
  c->deval.alloc(size_t(2) * P);
  c->deps.alloc(size_t(2) * P);
  c->dvalid.alloc(size_t(nk) * M);
  c->dstatus.alloc(nk);
  c->dchange.alloc(nk);
  // current / previous orbitals of the loop (right and left), and the mixed operator set
  c->dcur.alloc(2 * blk);
  c->dold.alloc(2 * blk);
  c->dnew.alloc(2 * blk);
  c->dmix.alloc(4 * blk);
  double* cur_r = c->dcur.p;
  double* cur_l = c->dcur.p + blk;
  double* old_r = c->dold.p;
  double* old_l = c->dold.p + blk;
  double* new_r = c->dnew.p;
  double* new_l = c->dnew.p + blk;
  double* mix_r = c->dmix.p;
  double* mix_l = c->dmix.p + 2 * blk;
  TC_HIP(hipMemcpyAsync(cur_r, sh.coef.p, blk * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (bitc) TC_HIP(hipMemcpyAsync(cur_l, sh.coefL.p, blk * sizeof(double), hipMemcpyDeviceToDevice, s));
  const double atol = 1e-8, rtol = 1e-8;
  double eprev = 0;
  int it = 0;
  bool mixed = false;
  for (; it < prm.max_iter; ++it) {
    TC_HIP(hipMemcpyAsync(c->dV.p, cur_r, blk * sizeof(double), hipMemcpyDeviceToDevice, s));
    TC_HIP(hipMemsetAsync(c->dvalid.p, 0, size_t(nk) * M * sizeof(int), s));
    hipLaunchKernelGGL(k_gram_schmidt, dim3(nk), dim3(256), 0, s, c->dV.p, c->dvalid.p, npwx, nk, nb, npm, M, 0,
                       nb, atol, rtol);
    for (int p = 0; p < nblk_sub; ++p) {
      if (p > 0) {
        hipLaunchKernelGGL(k_precond_residual, dim3(P), dim3(256), 0, s, c->dV.p, c->dHV.p, c->deps.p, kgx,
                           npwx, nk, nb, npm, p, atol);
        hipLaunchKernelGGL(k_gram_schmidt, dim3(nk), dim3(256), 0, s, c->dV.p, c->dvalid.p, npwx, nk, nb, npm,
                           M, p * nb, (p + 1) * nb, 0.0, rtol);
      }
      st = do_apply_vectors(c, nb, c->dV.p + p * blk, c->dHV.p + p * blk);
      if (st != TC_OK) return st;
      hipLaunchKernelGGL(k_add_kinetic, dim3(nblk(long(P) * npm)), dim3(256), 0, s, c->dV.p, c->dHV.p, kgx,
                         npwx, nk, nb, npm, p);
      if (p == 0)
        hipLaunchKernelGGL(k_rayleigh, dim3(P), dim3(256), 0, s, c->dV.p, c->dHV.p, npwx, nk, nb, npm,
                           c->deps.p);
    }
    hipLaunchKernelGGL(k_subspace_matrix, dim3(nk * M * M), dim3(256), 0, s, c->dV.p, c->dHV.p, npwx, nk, nb,
                       npm, M, c->dHs.p);
    hipLaunchKernelGGL(k_subspace_eig, dim3((nk + 63) / 64), dim3(64), 0, s, c->dHs.p, c->dvalid.p, nk, nb, M,
                       c->dwork.p, c->dX.p, c->dY.p, c->deval.p, c->dstatus.p, c->dchange.p);
    std::vector<int> status(nk);
    std::vector<double> change(nk);
    TC_HIP(hipMemcpyAsync(status.data(), c->dstatus.p, nk * sizeof(int), hipMemcpyDeviceToHost, s));
    TC_HIP(hipMemcpyAsync(change.data(), c->dchange.p, nk * sizeof(double), hipMemcpyDeviceToHost, s));
    TC_HIP(hipStreamSynchronize(s));
    double dmax = 0;
    for (int k = 0; k < nk; ++k) {
      if (status[k] == 1) return fail(c, TC_ERR_DEVICE, "subspace eigensolver did not converge");
      if (status[k] == 2) return fail(c, TC_ERR_ARG, "fewer independent trial vectors than bands");
      dmax = std::max(dmax, change[k]);
    }
    hipLaunchKernelGGL(k_subspace_combine, dim3(nblk(long(P) * npm)), dim3(256), 0, s, c->dV.p, c->dX.p, nk, nb,
                       npm, M, new_r);
    if (!bitc) {
      TC_HIP(hipMemsetAsync(c->dvalid.p, 0, size_t(nk) * M * sizeof(int), s));
      hipLaunchKernelGGL(k_gram_schmidt, dim3(nk), dim3(256), 0, s, new_r, c->dvalid.p, npwx, nk, nb, npm, M, 0,
                         nb, 0.0, 0.0);
    } else {
      hipLaunchKernelGGL(k_subspace_combine, dim3(nblk(long(P) * npm)), dim3(256), 0, s, c->dV.p, c->dY.p, nk, nb,
                         npm, M, new_l);
      sh.bo_l.alloc(kb);
      for (int k = 0; k < nk; ++k) {
        TC_HIP(hipMemcpyAsync(sh.bo_l.p, new_l + k * kb, kb * sizeof(double), hipMemcpyDeviceToDevice, s));
        st = biorthogonalize_at(c, k % pb.nk, nb, new_r + k * kb, new_l + k * kb);   // block k: channel k / nk
        if (st != TC_OK) return st;
      }
    }
    // previous <- current <- new
    TC_HIP(hipMemcpyAsync(c->dold.p, c->dcur.p, 2 * blk * sizeof(double), hipMemcpyDeviceToDevice, s));
    TC_HIP(hipMemcpyAsync(c->dcur.p, c->dnew.p, 2 * blk * sizeof(double), hipMemcpyDeviceToDevice, s));
    // operator of the next iteration: the new orbitals, or with mixing beta the new orbitals (beta f) and
    // the previous ones ((1 - beta) f) as extra bands (density-matrix mixing, Sec. 2.4)
    if (prm.mix < 1.0) {
      std::vector<double> fm(size_t(2) * P);
      for (int k = 0; k < nk; ++k)
        for (int side = 0; side < (bitc ? 2 : 1); ++side) {
          double* dst = side ? mix_l : mix_r;
          TC_HIP(hipMemcpyAsync(dst + 2 * k * kb, (side ? cur_l : cur_r) + k * kb, kb * sizeof(double),
                                hipMemcpyDeviceToDevice, s));
          TC_HIP(hipMemcpyAsync(dst + (2 * k + 1) * kb, (side ? old_l : old_r) + k * kb, kb * sizeof(double),
                                hipMemcpyDeviceToDevice, s));
        }
      for (int k = 0; k < nk; ++k)
        for (int i = 0; i < nb; ++i) {
          fm[size_t(k) * 2 * nb + i] = prm.mix * f[size_t(k) * nb + i];
          fm[size_t(k) * 2 * nb + nb + i] = (1.0 - prm.mix) * f[size_t(k) * nb + i];
        }
      load_set(c, mix_r, bitc ? mix_l : nullptr, 2 * nb, fm);
      mixed = true;
    } else {
      load_set(c, cur_r, bitc ? cur_l : nullptr, nb, f);
    }
    run_apply(c, nullptr, nullptr);
    if (ehist) ehist[it] = c->e_total;
    if (it > 0 && std::fabs(c->e_total - eprev) < prm.etol && (prm.otol <= 0 || dmax < prm.otol)) {
      ++it;
      break;
    }
    eprev = c->e_total;
  }
  if (mixed) {   // the context ends with the loop's orbitals alone and their energies
    load_set(c, cur_r, bitc ? cur_l : nullptr, nb, f);
    run_apply(c, nullptr, nullptr);
  }
  if (niter) *niter = it;
  return TC_OK;
}

// Orbitals of one spin channel at k-point ik to the host (tc_get_orbitals / tc_get_orbitals_spin).
int get_orbitals(tc_ctx* c, int spin, int ik, double* right, double* left) {
  Problem& pb = c->pb;
  if (ik < 0 || ik >= pb.nk) return fail(c, TC_ERR_ARG, "k-point index out of range");
  if (spin < 0 || spin >= pb.nspin) return fail(c, TC_ERR_ARG, "spin channel out of range");
  if (!(spin == 0 ? pb.loaded[ik] : pb.loaded_dn[ik])) return fail(c, TC_ERR_STATE, "orbitals of this k-point are not loaded");
  if (left && !(spin == 0 ? pb.left[ik] : pb.left_dn[ik]))
    return fail(c, TC_ERR_STATE, "no left orbitals on this k-point");
  const int nb = pb.nb, npw = pb.npw[ik], npm = pb.npw_max;
  std::vector<double> buf(size_t(2) * nb * npm);
  for (int side = 0; side < 2; ++side) {
    double* dst = side == 0 ? right : left;
    if (!dst) continue;
    const double* src = (side == 0 ? c->sh.coef.p : c->sh.coefL.p) + size_t(2) * (size_t(spin) * pb.nk + ik) * nb * npm;
    TC_HIP(hipMemcpy(buf.data(), src, buf.size() * sizeof(double), hipMemcpyDeviceToHost));
    for (int b = 0; b < nb; ++b)
      std::memcpy(dst + size_t(2) * b * npw, &buf[size_t(2) * b * npm], size_t(2) * npw * sizeof(double));
  }
  return TC_OK;
}

}  // namespace

extern "C" {

int tc_create(int device, void* stream, tc_ctx** out) {
  if (!out) return TC_ERR_ARG;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return TC_ERR_DEVICE;
  tc_ctx* c = new (std::nothrow) tc_ctx();
  if (!c) return TC_ERR_OOM;
  c->device = device;
  int st = guard(c, [&]() -> int {
    if (stream) {
      c->stream = reinterpret_cast<hipStream_t>(stream);
    } else {
      TC_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
      c->own_stream = true;
    }
    upload_twiddles();
    c->scratch = scratch_on(device);
    return TC_OK;
  });
  if (st != TC_OK) {
    delete c;
    return st;
  }
  *out = c;
  return TC_OK;
}

void tc_destroy(tc_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipStreamSynchronize(c->stream);
  c->eng.reset();
  if (c->own_stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

const char* tc_last_error(const tc_ctx* c) { return c ? c->err.c_str() : "null context"; }

int tc_set_cell(tc_ctx* c, const double lat[9]) {
  return guard_host(c, [&]() -> int {
    if (!lat) return fail(c, TC_ERR_ARG, "null lattice");
    Problem& pb = c->pb;
    const double* a = lat;
    const double det = a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
                       a[2] * (a[3] * a[7] - a[4] * a[6]);
    if (!(std::fabs(det) > 1e-12)) return fail(c, TC_ERR_ARG, "degenerate lattice");
    for (int i = 0; i < 9; ++i) pb.lat[i] = lat[i];
    pb.omega = std::fabs(det);
    // B = 2 pi inv(A)^T: rows b_j with a_i . b_j = 2 pi delta_ij
    const double inv[9] = {(a[4] * a[8] - a[5] * a[7]) / det, (a[2] * a[7] - a[1] * a[8]) / det,
                           (a[1] * a[5] - a[2] * a[4]) / det, (a[5] * a[6] - a[3] * a[8]) / det,
                           (a[0] * a[8] - a[2] * a[6]) / det, (a[2] * a[3] - a[0] * a[5]) / det,
                           (a[3] * a[7] - a[4] * a[6]) / det, (a[1] * a[6] - a[0] * a[7]) / det,
                           (a[0] * a[4] - a[1] * a[3]) / det};
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) pb.B[3 * j + k] = 2.0 * kPi * inv[3 * k + j];
    pb.cell = true;
    pb.nsym = 0;   // operations are stated for a given cell, k-mesh and grid
    pb.band_alpha = -1;
    c->tables_dirty = true;
    c->have_result = false;
    return TC_OK;
  });
}

int tc_set_kmesh(tc_ctx* c, int n1, int n2, int n3) {
  return guard_host(c, [&]() -> int {
    if (n1 < 1 || n2 < 1 || n3 < 1 || n1 > 16 || n2 > 16 || n3 > 16) return fail(c, TC_ERR_KMESH, "k-mesh out of range");
    Problem& pb = c->pb;
    pb.n1 = n1;
    pb.n2 = n2;
    pb.n3 = n3;
    pb.nk = n1 * n2 * n3;
    pb.kshift[0] = pb.kshift[1] = pb.kshift[2] = 0.0;
    pb.miller.assign(pb.nk, {});
    pb.npw.assign(pb.nk, 0);
    pb.loaded.assign(pb.nk, 0);
    pb.left.assign(pb.nk, 0);
    pb.loaded_dn.assign(pb.nk, 0);
    pb.left_dn.assign(pb.nk, 0);
    pb.nb = 0;
    pb.nsym = 0;
    pb.nkb = 0;   // band k-points are coded after the mesh ones
    c->tables_dirty = true;
    c->have_result = false;
    return TC_OK;
  });
}

int tc_set_grid(tc_ctx* c, int N1, int N2, int N3) {
  return guard_host(c, [&]() -> int {
    if (N1 != N2 || N2 != N3 || !grid_supported(N1))
      return fail(c, TC_ERR_UNSUPPORTED, "only cubic grids N^3 with N in {8,12,16,24,32,48} are built");
    c->pb.N = N1;
    c->pb.nsym = 0;
    c->tables_dirty = true;
    c->have_result = false;
    return TC_OK;
  });
}

int tc_set_basis(tc_ctx* c, int ik, int npw, const int32_t* miller) {
  return guard_host(c, [&]() -> int {
    Problem& pb = c->pb;
    if (pb.nk == 0 || pb.N == 0) return fail(c, TC_ERR_STATE, "set the k-mesh and grid first");
    if (ik < 0 || ik >= pb.nk || npw <= 0 || !miller) return fail(c, TC_ERR_ARG, "bad basis arguments");
    for (int g = 0; g < 3 * npw; ++g)
      if (miller[g] >= pb.N / 2 || miller[g] < -(pb.N / 2) + 1)
        return fail(c, TC_ERR_GRID, "plane wave outside the FFT grid");
    std::vector<char> seen(size_t(pb.N) * pb.N * pb.N, 0);   // two coefficients on one grid point
    for (int g = 0; g < npw; ++g) {
      size_t idx = 0;
      for (int d = 0; d < 3; ++d) idx = idx * pb.N + size_t((miller[3 * g + d] + pb.N) % pb.N);
      if (seen[idx]) return fail(c, TC_ERR_ARG, "plane wave listed twice in the basis");
      seen[idx] = 1;
    }
    pb.miller[ik].assign(miller, miller + 3 * npw);
    pb.npw[ik] = npw;
    pb.loaded[ik] = 0;
    pb.sym_ready = false;
    c->have_result = false;
    return TC_OK;
  });
}

int tc_set_jastrow(tc_ctx* c, const double A[2], const double C[2]) {
  return guard_host(c, [&]() -> int {
    if (!A || !C) return fail(c, TC_ERR_ARG, "null Jastrow parameters");
    for (int i = 0; i < 2; ++i)
      if (!(A[i] >= 0.0) || !(C[i] > 0.0)) return fail(c, TC_ERR_ARG, "need A >= 0 and C > 0");
    for (int i = 0; i < 2; ++i) {
      c->pb.A[i] = A[i];
      c->pb.C[i] = C[i];
    }
    c->pb.jastrow = true;
    c->tables_dirty = true;
    c->have_result = false;
    return TC_OK;
  });
}

int tc_set_kmesh_shift(tc_ctx* c, const double shift[3]) {
  return guard_host(c, [&]() -> int {
    Problem& pb = c->pb;
    if (pb.nk == 0) return fail(c, TC_ERR_STATE, "set the k-mesh before its shift");
    if (!shift) return fail(c, TC_ERR_ARG, "null shift");
    for (int i = 0; i < 3; ++i)
      if (!(shift[i] >= 0.0 && shift[i] < 1.0)) return fail(c, TC_ERR_ARG, "shift components must lie in [0, 1)");
    for (int i = 0; i < 3; ++i) pb.kshift[i] = shift[i];
    // the k-points moved: orbitals and symmetry are set again (the plane-wave sets are the caller's)
    std::fill(pb.loaded.begin(), pb.loaded.end(), 0);
    std::fill(pb.left.begin(), pb.left.end(), 0);
    std::fill(pb.loaded_dn.begin(), pb.loaded_dn.end(), 0);
    std::fill(pb.left_dn.begin(), pb.left_dn.end(), 0);
    pb.nsym = 0;
    pb.sym_ready = false;
    c->tables_dirty = true;
    c->have_result = false;
    return TC_OK;
  });
}

int tc_set_jastrow_cusp(tc_ctx* c, const double A[2]) {
  return guard_host(c, [&]() -> int {
    if (!A) return fail(c, TC_ERR_ARG, "null Jastrow parameters");
    for (int i = 0; i < 2; ++i)
      if (!(A[i] > 0.0)) return fail(c, TC_ERR_ARG, "the cusp conditions need A > 0");
    // Eq. cusp: C = sqrt(2 A) for parallel spins, sqrt(A) for antiparallel ones
    c->pb.A[0] = A[0];
    c->pb.A[1] = A[1];
    c->pb.C[0] = std::sqrt(2.0 * A[0]);
    c->pb.C[1] = std::sqrt(A[1]);
    c->pb.jastrow = true;
    c->tables_dirty = true;
    c->have_result = false;
    return TC_OK;
  });
}

int tc_set_options(tc_ctx* c, int precision, double alpha, int div_correction, uint64_t term_mask) {
  return guard_host(c, [&]() -> int {
    if (precision != TC_PREC_FP64 && precision != TC_PREC_FP32 && precision != TC_PREC_FP32_SPLITBF16)
      return fail(c, TC_ERR_ARG, "unknown precision");
    if (!(alpha > 0.0)) return fail(c, TC_ERR_ARG, "alpha must be > 0");
    if (div_correction != TC_DIV_OFF && div_correction != TC_DIV_PRINTED && div_correction != TC_DIV_LIMIT)
      return fail(c, TC_ERR_ARG, "div_correction must be TC_DIV_OFF, TC_DIV_PRINTED or TC_DIV_LIMIT");
    Problem& pb = c->pb;
    pb.prec = precision;
    pb.alpha = alpha;
    pb.div = div_correction != TC_DIV_OFF;
    pb.reading = div_correction == TC_DIV_LIMIT ? TC_DIV_LIMIT : TC_DIV_PRINTED;
    pb.mask = term_mask & TC_T_ALL;
    pb.options = true;
    c->tables_dirty = true;
    c->have_result = false;
    return TC_OK;
  });
}

int tc_load_orbitals(tc_ctx* c, int ik, int nband, const double* right, const double* left, const double* occ) {
  return guard(c, [&]() -> int {
    if (!right) return fail(c, TC_ERR_ARG, "null coefficients");
    int st = begin_load(c, ik, nband, occ);
    if (st != TC_OK) return st;
    Problem& pb = c->pb;
    const int npw = pb.npw[ik];
    pb.loaded[ik] = 0;
    pb.left[ik] = 0;
    c->have_result = false;
    std::vector<double> stage(size_t(2) * nband * pb.npw_max, 0.0);
    auto pack = [&](const double* src) {
      for (int b = 0; b < nband; ++b)
        std::memcpy(&stage[size_t(2) * b * pb.npw_max], src + size_t(2) * b * npw, size_t(2) * npw * sizeof(double));
    };
    pack(right);
    TC_HIP(hipMemcpy(c->sh.coef.p + size_t(2) * ik * nband * pb.npw_max, stage.data(), stage.size() * sizeof(double),
                     hipMemcpyHostToDevice));
    upload_basis_data(c);
    if (left) {
      pack(left);
      c->sh.bo_l.alloc(stage.size());
      TC_HIP(hipMemcpy(c->sh.bo_l.p, stage.data(), stage.size() * sizeof(double), hipMemcpyHostToDevice));
      st = biorthogonalize(c, ik);
      if (st != TC_OK) return st;
      pb.left[ik] = 1;
    }
    pb.loaded[ik] = 1;
    return TC_OK;
  });
}

int tc_set_nspin(tc_ctx* c, int nspin) {
  return guard_host(c, [&]() -> int {
    if (nspin != 1 && nspin != 2) return fail(c, TC_ERR_ARG, "nspin must be 1 or 2");
    Problem& pb = c->pb;
    if (pb.nk == 0) return fail(c, TC_ERR_STATE, "set the k-mesh before the number of spin channels");
    pb.nspin = nspin;
    pb.nb = 0;   // every channel is loaded again
    std::fill(pb.loaded.begin(), pb.loaded.end(), 0);
    std::fill(pb.left.begin(), pb.left.end(), 0);
    pb.loaded_dn.assign(pb.nk, 0);
    pb.left_dn.assign(pb.nk, 0);
    c->have_result = false;
    return TC_OK;
  });
}

int tc_set_band_kpoints(tc_ctx* c, int nkb, const double* kfrac) {
  return guard_host(c, [&]() -> int { return set_band_kpoints(c, nkb, kfrac); });
}

int tc_set_band_basis(tc_ctx* c, int ib, int npw, const int32_t* miller) {
  return guard_host(c, [&]() -> int { return set_band_basis(c, ib, npw, miller); });
}

int tc_load_band_orbitals(tc_ctx* c, int ib, int nband, const double* coef, const double* occ) {
  return guard(c, [&]() -> int { return load_band_orbitals(c, ib, nband, coef, occ); });
}

int tc_apply_band(tc_ctx* c, double* out, double* eps) {
  return guard(c, [&]() -> int { return do_apply_band(c, out, eps); });
}

int tc_set_symmetry(tc_ctx* c, int nsym, const int32_t* rot, const double* tau) {
  return guard_host(c, [&]() -> int { return set_symmetry(c, nsym, rot, tau); });
}

int tc_load_orbitals_spin(tc_ctx* c, int spin, int ik, int nband, const double* right, const double* left,
                          const double* occ) {
  if (spin == 0) return tc_load_orbitals(c, ik, nband, right, left, occ);
  return guard(c, [&]() -> int {
    Problem& pb = c->pb;
    if (spin != 1) return fail(c, TC_ERR_ARG, "spin must be 0 or 1");
    if (pb.nspin != 2) return fail(c, TC_ERR_STATE, "tc_set_nspin(ctx, 2) first");
    if (!right) return fail(c, TC_ERR_ARG, "null coefficients");
    int st = begin_load(c, ik, nband, occ, 1);
    if (st != TC_OK) return st;
    const int npw = pb.npw[ik];
    pb.loaded_dn[ik] = 0;
    pb.left_dn[ik] = 0;
    c->have_result = false;
    std::vector<double> stage(size_t(2) * nband * pb.npw_max, 0.0);
    auto pack = [&](const double* src) {
      for (int b = 0; b < nband; ++b)
        std::memcpy(&stage[size_t(2) * b * pb.npw_max], src + size_t(2) * b * npw, size_t(2) * npw * sizeof(double));
    };
    pack(right);
    const size_t off = size_t(2) * (pb.P() + size_t(ik) * nband) * pb.npw_max;   // channel 1, k-point ik
    TC_HIP(hipMemcpy(c->sh.coef.p + off, stage.data(), stage.size() * sizeof(double), hipMemcpyHostToDevice));
    upload_basis_data(c);
    if (left) {   // biorthogonalised within the channel, as for channel 0
      pack(left);
      c->sh.bo_l.alloc(stage.size());
      TC_HIP(hipMemcpy(c->sh.bo_l.p, stage.data(), stage.size() * sizeof(double), hipMemcpyHostToDevice));
      c->sh.coefL.alloc(size_t(2) * pb.nspin * pb.P() * pb.npw_max);
      st = biorthogonalize_at(c, ik, nband, c->sh.coef.p + off, c->sh.coefL.p + off);
      if (st != TC_OK) return st;
      pb.left_dn[ik] = 1;
    }
    pb.loaded_dn[ik] = 1;
    return TC_OK;
  });
}

int tc_load_orbitals_dev(tc_ctx* c, int ik, int nband, const void* right_dev, const double* occ) {
  return guard(c, [&]() -> int {
    if (!right_dev) return fail(c, TC_ERR_ARG, "null coefficients");
    int st = begin_load(c, ik, nband, occ);
    if (st != TC_OK) return st;
    Problem& pb = c->pb;
    const int npw = pb.npw[ik];
    double* dst = c->sh.coef.p + size_t(2) * ik * nband * pb.npw_max;
    TC_HIP(hipMemsetAsync(dst, 0, size_t(2) * nband * pb.npw_max * sizeof(double), c->stream));
    TC_HIP(hipMemcpy2DAsync(dst, size_t(2) * pb.npw_max * sizeof(double), right_dev, size_t(2) * npw * sizeof(double),
                            size_t(2) * npw * sizeof(double), nband, hipMemcpyDeviceToDevice, c->stream));
    TC_HIP(hipStreamSynchronize(c->stream));
    pb.loaded[ik] = 1;
    pb.left[ik] = 0;
    upload_basis_data(c);
    c->have_result = false;
    return TC_OK;
  });
}

int tc_apply_all(tc_ctx* c, double* out) {
  return guard(c, [&]() -> int { return do_apply(c, nullptr, out); });
}

int tc_apply_all_dev(tc_ctx* c, void* out_dev) {
  return guard(c, [&]() -> int { return do_apply(c, out_dev, nullptr); });
}

int tc_apply_all_dev_noalloc(tc_ctx* c, void* out_dev) {
  return guard(c, [&]() -> int { return do_apply_noalloc(c, out_dev); });
}

int tc_scf(tc_ctx* c, const tc_scf_params* prm, double* energies, int* iterations) {
  return guard(c, [&]() -> int {
    if (!prm) return fail(c, TC_ERR_ARG, "null parameters");
    return do_scf(c, *prm, energies, iterations);
  });
}

int tc_get_orbitals_spin(tc_ctx* c, int spin, int ik, double* right, double* left) {
  return guard(c, [&]() -> int { return get_orbitals(c, spin, ik, right, left); });
}

int tc_get_orbitals(tc_ctx* c, int ik, double* right, double* left) {
  return guard(c, [&]() -> int {
    Problem& pb = c->pb;
    if (ik < 0 || ik >= pb.nk) return fail(c, TC_ERR_ARG, "k-point index out of range");
    if (!pb.loaded[ik]) return fail(c, TC_ERR_STATE, "orbitals of this k-point are not loaded");
    if (left && !pb.left[ik]) return fail(c, TC_ERR_STATE, "no left orbitals on this k-point");
    const int nb = pb.nb, npw = pb.npw[ik], npm = pb.npw_max;
    std::vector<double> buf(size_t(2) * nb * npm);
    for (int side = 0; side < 2; ++side) {
      double* dst = side == 0 ? right : left;
      if (!dst) continue;
      const double* src = (side == 0 ? c->sh.coef.p : c->sh.coefL.p) + size_t(2) * ik * nb * npm;
      TC_HIP(hipMemcpy(buf.data(), src, buf.size() * sizeof(double), hipMemcpyDeviceToHost));
      for (int b = 0; b < nb; ++b)
        std::memcpy(dst + size_t(2) * b * npw, &buf[size_t(2) * b * npm], size_t(2) * npw * sizeof(double));
    }
    return TC_OK;
  });
}

int tc_apply(tc_ctx* c, int nvec, const double* in, double* out) {
  return guard(c, [&]() -> int {
    if (!in || !out) return fail(c, TC_ERR_ARG, "null vectors");
    if (nvec <= 0) return fail(c, TC_ERR_ARG, "nvec must be positive");
    int st = prepare(c);
    if (st != TC_OK) return st;
    const size_t n = size_t(2) * c->pb.nspin * c->pb.nk * nvec * c->pb.npw_max;
    c->coefT.alloc(n);
    c->outT.alloc(n);
    TC_HIP(hipMemcpy(c->coefT.p, in, n * sizeof(double), hipMemcpyHostToDevice));
    st = do_apply_vectors(c, nvec, c->coefT.p, c->outT.p);
    if (st != TC_OK) return st;
    TC_HIP(hipMemcpy(out, c->outT.p, n * sizeof(double), hipMemcpyDeviceToHost));
    return TC_OK;
  });
}

int tc_apply_dev(tc_ctx* c, int nvec, const void* in_dev, void* out_dev) {
  return guard(c, [&]() -> int {
    if (!in_dev || !out_dev) return fail(c, TC_ERR_ARG, "null vectors");
    return do_apply_vectors(c, nvec, static_cast<const double*>(in_dev), static_cast<double*>(out_dev));
  });
}

int tc_orbital_energies(tc_ctx* c, double* eps) {
  return guard(c, [&]() -> int {
    if (!eps) return fail(c, TC_ERR_ARG, "null output");
    if (!c->have_result) {
      int st = do_apply(c, nullptr, nullptr);
      if (st != TC_OK) return st;
    }
    std::memcpy(eps, c->eps.data(), c->eps.size() * sizeof(double));
    return TC_OK;
  });
}

int tc_energy(tc_ctx* c, double* e_total, double* e_parts) {
  return guard(c, [&]() -> int {
    if (!c->have_result) {
      int st = do_apply(c, nullptr, nullptr);
      if (st != TC_OK) return st;
    }
    if (e_total) *e_total = c->e_total;
    if (e_parts)
      for (int i = 0; i < TC_E_NPARTS; ++i) e_parts[i] = c->e_parts[i];
    return TC_OK;
  });
}

int tc_energy_backward(tc_ctx* c, double* grad, double dA[2], double dC[2]) {
  return guard(c, [&]() -> int {
    if (!grad && !dA && !dC) return fail(c, TC_ERR_ARG, "nothing requested");
    int st = prepare(c);
    if (st != TC_OK) return st;
    if (c->pb.bitc && grad)
      return fail(c, TC_ERR_UNSUPPORTED, "left orbitals loaded: use tc_energy_backward_lr for the two gradients");
    return do_backward(c, nullptr, grad, dA, dC);
  });
}

int tc_energy_backward_lr(tc_ctx* c, double* grad_right, double* grad_left, double dA[2], double dC[2]) {
  return guard(c, [&]() -> int {
    if (!grad_right && !grad_left && !dA && !dC) return fail(c, TC_ERR_ARG, "nothing requested");
    return do_backward(c, nullptr, grad_right, dA, dC, nullptr, grad_left);
  });
}

int tc_energy_backward_dev(tc_ctx* c, void* grad_dev, double dA[2], double dC[2]) {
  return guard(c, [&]() -> int {
    if (!grad_dev && !dA && !dC) return fail(c, TC_ERR_ARG, "nothing requested");
    int st = prepare(c);
    if (st != TC_OK) return st;
    if (c->pb.bitc && grad_dev)
      return fail(c, TC_ERR_UNSUPPORTED, "left orbitals loaded: use tc_energy_backward_lr for the two gradients");
    return do_backward(c, grad_dev, nullptr, dA, dC);
  });
}

int tc_sync(tc_ctx* c) {
  return guard(c, [&]() -> int {
    TC_HIP(hipStreamSynchronize(c->stream));
    return TC_OK;
  });
}

int tc_set_batch(tc_ctx* c, int targets_per_batch) {
  return guard_host(c, [&]() -> int {
    if (targets_per_batch < 0) return fail(c, TC_ERR_ARG, "batch must be >= 0");
    c->pb.batch = targets_per_batch;
    c->have_result = false;
    return TC_OK;
  });
}

int tc_set_pair_store(tc_ctx* c, int on) {
  return guard(c, [&]() -> int {
    c->pb.pair_store = on != 0;
    if (!on && c->eng) {   // release now (the stream's queued work may still read it)
      TC_HIP(hipStreamSynchronize(c->stream));
      c->eng->release_pair_store();
    }
    c->have_result = false;
    return TC_OK;
  });
}

int tc_set_allocator(tc_ctx* c, void* (*alloc_fn)(size_t, void*), void (*free_fn)(void*, size_t, void*), void* user) {
  return guard(c, [&]() -> int {
    if ((alloc_fn == nullptr) != (free_fn == nullptr))
      return fail(c, TC_ERR_ARG, "give both an allocation and a release function, or neither");
    if (!alloc_fn) {
      c->cur_alloc = nullptr;
      return TC_OK;
    }
    c->allocs.push_back(DevAlloc{alloc_fn, free_fn, user, c->stream});
    c->cur_alloc = &c->allocs.back();
    return TC_OK;
  });
}

int tc_set_memory_budget(tc_ctx* c, size_t bytes) {
  return guard_host(c, [&]() -> int {
    c->pb.mem_budget = bytes;
    return TC_OK;
  });
}

void* tc_get_stream(const tc_ctx* c) { return c ? reinterpret_cast<void*>(c->stream) : nullptr; }

int tc_set_profiling(tc_ctx* c, int on) {
  return guard_host(c, [&]() -> int {
    c->prof.on = on != 0;
    return TC_OK;
  });
}

int tc_kernel_stats(tc_ctx* c, double* ms, double* launches, double* bytes, int reset) {
  return guard(c, [&]() -> int {
    for (int i = 0; i < TC_K_NKERNEL; ++i) {
      if (ms) ms[i] = c->prof.ms[i];
      if (launches) launches[i] = c->prof.launches[i];
      if (bytes) bytes[i] = c->prof.bytes[i];
    }
    if (reset) c->prof.reset();
    return TC_OK;
  });
}

int tc_last_timing(tc_ctx* c, double* total_ms, double* stage_ms, int n) {
  return guard(c, [&]() -> int {
    if (total_ms) *total_ms = c->total_ms;
    for (int i = 0; i < n && i < 6; ++i)
      if (stage_ms) stage_ms[i] = c->stage_ms[i];
    return TC_OK;
  });
}

}  // extern "C"
