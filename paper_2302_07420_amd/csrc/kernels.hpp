// Device kernels of the transcorrelated-operator path (gfx950).
//
// Field layout: one complex field on the N^3 grid is [z][y][x] with x fastest;
// x, y, z run along a1, a2, a3 and hold Miller index m = i (i < N/2) or i - N.
// A batch of fields is contiguous ([field][N^3]).  Fields of the pair passes
// are indexed pair-major: pair (t, q) = t*P + q, then component.
//
// Units: orbitals are stored as psi = sqrt(Omega) * (cell-periodic part) (the
// paper's dimensionless arrays, Sec. 2.6.1).  Every kernel table is stored
// multiplied by 1/(Omega N^3), so that for a source that is a product of two
// such orbitals (times physical potentials), IFFT[K_table * FFT(source)] is the
// physical convolution sum_G K(Delta+G) FT[source_phys](G) e^{iG.r}.
#pragma once
#include "fft_reg.hpp"
#include "reduce.hpp"
#include <hip/hip_bf16.h>

namespace tcmi {

struct Recip {
  double b[9];   // rows b1, b2, b3 (cartesian, bohr^-1)
};

struct MeshInfo {
  int n1, n2, n3;   // k-mesh
  int nb;           // bands per k-point of the occupied (partner) set
  int P;            // orbitals of one spin channel (nk * nb)
  int nbt;          // vectors per k-point of the target set (nb when the targets are the orbitals)
  const int* tk = nullptr;   // k-point of target block j / nbt (device; null: the block index itself)
  int nkb = 0;               // band k-points, coded nk .. nk + nkb - 1 in tk
  int qoff = 0;              // partner q of a pass is orbital q + qoff (a pass over partners qoff .. P - 1)
  int trq = 0;               // z stage: > 0, the rows of a triangular store with Q1 = trq (pair_tq)
};

__device__ __forceinline__ int kindex_delta(const MeshInfo& mi, int kto, int kfrom) {
  // index of Delta = k_to - k_from (fractions (i_to - i_from)/n) in [0, prod(2n-1))
  const int a3 = kto % mi.n3, a2 = (kto / mi.n3) % mi.n2, a1 = kto / (mi.n3 * mi.n2);
  const int b3 = kfrom % mi.n3, b2 = (kfrom / mi.n3) % mi.n2, b1 = kfrom / (mi.n3 * mi.n2);
  return ((a1 - b1 + mi.n1 - 1) * (2 * mi.n2 - 1) + (a2 - b2 + mi.n2 - 1)) * (2 * mi.n3 - 1) + (a3 - b3 + mi.n3 - 1);
}

template <int N>
__device__ __forceinline__ int mfreq(int i) { return i < N / 2 ? i : i - N; }

// cartesian Q = (delta + m) . B for grid point (x, y, z)
template <typename R, int N>
__device__ __forceinline__ void qvec(const Recip& rc, const double* dfr, int x, int y, int z, R* Q) {
  const double f1 = dfr[0] + mfreq<N>(x), f2 = dfr[1] + mfreq<N>(y), f3 = dfr[2] + mfreq<N>(z);
#pragma unroll
  for (int c = 0; c < 3; ++c) Q[c] = R(f1 * rc.b[c] + f2 * rc.b[3 + c] + f3 * rc.b[6 + c]);
}

// ---------------------------------------------------------------- plane count per xy block
template <typename R, int N>
struct XY {
  static constexpr int kLdsBudget = 65536;
  static constexpr int kByLds = kLdsBudget / int(N * (N + 1) * sizeof(cx<R>));
  static constexpr int kByThr = 256 / N;
  static constexpr int PB = (kByLds < kByThr ? kByLds : kByThr) < 1 ? 1 : (kByLds < kByThr ? kByLds : kByThr);
  static constexpr int THREADS = PB * N;
};

// Generic 2D transform of planes.  LOAD(plane, y, x) returns the input element,
// STORE(plane, y, x, v) consumes the output; the plane loop is coalesced on x.
template <typename R, int N, int DIR, class IO>
__device__ __forceinline__ void xy_block(IO& io, long nplanes) {
  constexpr int PB = XY<R, N>::PB;
  constexpr int LD = N + 1;
  __shared__ cx<R> sm[PB * N * LD];
  const int tid = threadIdx.x;
  const long p0 = long(blockIdx.x) * PB;
  const int np = int(nplanes - p0 < PB ? nplanes - p0 : PB);
  for (int e = tid; e < np * N * N; e += PB * N) {
    const int p = e / (N * N), rem = e - p * N * N, y = rem / N, x = rem - y * N;
    sm[(p * N + y) * LD + x] = io.load(p0 + p, y, x);
  }
  __syncthreads();
  const int p = tid / N, l = tid - (tid / N) * N;
  cx<R> v[N];
  if (p < np) {
#pragma unroll
    for (int x = 0; x < N; ++x) v[x] = sm[(p * N + l) * LD + x];
    fft_line<R, N, DIR>(v);
#pragma unroll
    for (int x = 0; x < N; ++x) sm[(p * N + l) * LD + x] = v[x];
  }
  __syncthreads();
  if (p < np) {
#pragma unroll
    for (int y = 0; y < N; ++y) v[y] = sm[(p * N + y) * LD + l];
    fft_line<R, N, DIR>(v);
#pragma unroll
    for (int y = 0; y < N; ++y) io.store(p0 + p, y, l, v[y]);
  }
}

template <typename R, int N>
struct IOPlain {
  cx<R>* d;
  __device__ cx<R> load(long pl, int y, int x) const { return d[pl * N * N + y * N + x]; }
  __device__ void store(long pl, int y, int x, cx<R> v) const { d[pl * N * N + y * N + x] = v; }
};

template <typename R, int N, int DIR>
__global__ void __launch_bounds__(256) k_fft_xy(cx<R>* d, long nplanes) {
  IOPlain<R, N> io{d};
  xy_block<R, N, DIR>(io, nplanes);
}

// z transform, one thread per column (vol, y, x)
template <typename R, int N, int DIR>
__global__ void __launch_bounds__(256) k_fft_z(cx<R>* d, long nvol) {
  const long col = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (col >= nvol * N * N) return;
  const long vol = col / (N * N);
  const int xy = int(col - vol * N * N);
  cx<R>* b = d + vol * N * N * N + xy;
  cx<R> v[N];
#pragma unroll
  for (int z = 0; z < N; ++z) v[z] = b[z * N * N];
  fft_line<R, N, DIR>(v);
#pragma unroll
  for (int z = 0; z < N; ++z) b[z * N * N] = v[z];
}

// ---------------------------------------------------------------- G -> r of orbitals
// out[p][box(g)] = c_p(g) (comp < 0) or i (k+G)_comp c_p(g); out zeroed beforehand.
template <typename R>
__global__ void k_scatter(const double* coef, const int* boxidx, const int* npw, const double* kg, int nb,
                          int npw_max, int P, int comp, cx<R>* out, long nr) {
  const long t = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= long(P) * npw_max) return;
  const int p = int(t / npw_max), g = int(t - long(p) * npw_max);
  const int ik = p / nb;
  if (g >= npw[ik]) return;
  double cr = coef[2 * t], ci = coef[2 * t + 1];
  if (comp >= 0) {
    const double q = kg[(long(ik) * npw_max + g) * 3 + comp];
    const double tr = -q * ci, ti = q * cr;
    cr = tr;
    ci = ti;
  }
  out[long(p) * nr + boxidx[long(ik) * npw_max + g]] = mk<R>(R(cr), R(ci));
}

// r -> G of per-target fields: out[j][g] (complex128) = field_j(box(g)) * scale, zero beyond npw
template <typename R>
__global__ void k_gather(const cx<R>* f, const int* boxidx, const int* npw, int nb, int npw_max, int j0, int nt,
                         double scale, double* out, long nr, const int* kmap = nullptr, int add = 0) {
  const long t = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= long(nt) * npw_max) return;
  const int jt = int(t / npw_max), g = int(t - long(jt) * npw_max);
  const int j = j0 + jt;
  const int ik = kmap ? kmap[j / nb] : j / nb;   // kmap: k-point of target block j / nb
  double re = 0, im = 0;
  if (g < npw[ik]) {
    const cx<R> v = f[long(jt) * nr + boxidx[long(ik) * npw_max + g]];
    re = double(v.x) * scale;
    im = double(v.y) * scale;
  }
  if (add) {   // accumulate onto what an earlier gather wrote
    re += out[2 * (long(j) * npw_max + g)];
    im += out[2 * (long(j) * npw_max + g) + 1];
  }
  out[2 * (long(j) * npw_max + g)] = re;
  out[2 * (long(j) * npw_max + g) + 1] = im;
}

// ---------------------------------------------------------------- densities
// n = sum_q w_q conj(chi_q) psi_q, J_c = sum_q w_q conj(chi_q) D_qc, accumulated in FP64 (Sec. 2.6.3;
// TC mode: chi = psi, the same array, and n is real).
template <typename R, int N>
__global__ void k_density(const cx<R>* chi, const cx<R>* psi, const cx<R>* D, const double* w, int P, cx<R>* n,
                          cx<R>* J) {
  constexpr long NR = long(N) * N * N;
  const long r = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= NR) return;
  const bool tc = chi == psi;
  double nn = 0, ni = 0, jr[3] = {0, 0, 0}, ji[3] = {0, 0, 0};
  for (int q = 0; q < P; ++q) {
    const cx<R> a = chi[q * NR + r];
    const double wq = w[q];
    if (tc) {
      nn += wq * (double(a.x) * a.x + double(a.y) * a.y);
    } else {
      const cx<R> b = psi[q * NR + r];
      nn += wq * (double(a.x) * b.x + double(a.y) * b.y);
      ni += wq * (double(a.x) * b.y - double(a.y) * b.x);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const cx<R> d = D[(long(c) * P + q) * NR + r];
      jr[c] += wq * (double(a.x) * d.x + double(a.y) * d.y);
      ji[c] += wq * (double(a.x) * d.y - double(a.y) * d.x);
    }
  }
  n[r] = mk<R>(R(nn), R(ni));
#pragma unroll
  for (int c = 0; c < 3; ++c) J[c * NR + r] = mk<R>(R(jr[c]), R(ji[c]));
}

// Hartree-type fields in G space (Delta = 0, G = 0 dropped through the tables):
// VH~ = V(G) n~, h1~_c = i G_c u(G) n~, P~ = -i G . u(G) J~  (V, u summed over both spin channels)
template <typename R, int N>
__global__ void k_hartree_g(const Recip rc, const R* tV, const R* tU, const cx<R>* nG, const cx<R>* JG,
                            cx<R>* out /* 5 vols: VH, h1 x3, P */) {
  constexpr long NR = long(N) * N * N;
  const long r = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= NR) return;
  const int x = int(r % N), y = int((r / N) % N), z = int(r / (N * N));
  const double zero[3] = {0, 0, 0};
  R Q[3];
  qvec<R, N>(rc, zero, x, y, z, Q);
  const cx<R> nn = nG[r];
  const R V = tV[r], U = tU[r];
  out[r] = V * nn;
  cx<R> p = mk<R>(R(0), R(0));
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    out[(1 + c) * NR + r] = mul_i((Q[c] * U) * nn);
    p = p + mul_i((-Q[c] * U) * JG[c * NR + r]);
  }
  out[4 * NR + r] = p;
}

// out~ = sum_c -i G_c u(G) in~_c (Delta = 0)
template <typename R, int N>
__global__ void k_gdiv(const Recip rc, const R* tU, const cx<R>* in, cx<R>* out) {
  constexpr long NR = long(N) * N * N;
  const long r = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= NR) return;
  const int x = int(r % N), y = int((r / N) % N), z = int(r / (N * N));
  const double zero[3] = {0, 0, 0};
  R Q[3];
  qvec<R, N>(rc, zero, x, y, z, Q);
  const R U = tU[r];
  cx<R> p = mk<R>(R(0), R(0));
#pragma unroll
  for (int c = 0; c < 3; ++c) p = p + mul_i((-Q[c] * U) * in[c * NR + r]);
  out[r] = p;
}

// src_c = h1_c * n
template <typename R, int N>
__global__ void k_mul_vec_scalar(const cx<R>* v, const cx<R>* s, cx<R>* out) {
  constexpr long NR = long(N) * N * N;
  const long r = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= NR) return;
#pragma unroll
  for (int c = 0; c < 3; ++c) out[c * NR + r] = v[c * NR + r] * s[r];
}

// Spin-polarised Hartree-type fields for target spin s: the parallel-channel kernels act on the own
// spin's densities (nG, JG), the antiparallel ones on the other spin's (nGo, JGo).
//   out: VH~, h1~ x3, P~ (as k_hartree_g)
template <typename R, int N>
__global__ void k_hartree_g2(const Recip rc, const R* tVp, const R* tVa, const R* tUp, const R* tUa, const cx<R>* nG,
                             const cx<R>* JG, const cx<R>* nGo, const cx<R>* JGo, cx<R>* out) {
  constexpr long NR = long(N) * N * N;
  const long r = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= NR) return;
  const int x = int(r % N), y = int((r / N) % N), z = int(r / (N * N));
  const double zero[3] = {0, 0, 0};
  R Q[3];
  qvec<R, N>(rc, zero, x, y, z, Q);
  const cx<R> n1 = nG[r], n2 = nGo[r];
  out[r] = tVp[r] * n1 + tVa[r] * n2;
  const cx<R> un = tUp[r] * n1 + tUa[r] * n2;
  cx<R> p = mk<R>(R(0), R(0));
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    out[(1 + c) * NR + r] = mul_i(Q[c] * un);
    p = p + mul_i((-Q[c]) * (tUp[r] * JG[c * NR + r] + tUa[r] * JGo[c * NR + r]));
  }
  out[4 * NR + r] = p;
}

// out~ = sum_c -i G_c (u_par in~_c + u_anti ino~_c)  (spin-polarised form of k_gdiv)
template <typename R, int N>
__global__ void k_gdiv2(const Recip rc, const R* tUp, const R* tUa, const cx<R>* in, const cx<R>* ino, cx<R>* out) {
  constexpr long NR = long(N) * N * N;
  const long r = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= NR) return;
  const int x = int(r % N), y = int((r / N) % N), z = int(r / (N * N));
  const double zero[3] = {0, 0, 0};
  R Q[3];
  qvec<R, N>(rc, zero, x, y, z, Q);
  cx<R> p = mk<R>(R(0), R(0));
#pragma unroll
  for (int c = 0; c < 3; ++c) p = p + mul_i((-Q[c]) * (tUp[r] * in[c * NR + r] + tUa[r] * ino[c * NR + r]));
  out[r] = p;
}

// h6 of target spin s (Alg. 3a2, spin-polarised): sum over own-spin partners of the parallel-channel h5
// and over other-spin partners of the antiparallel-channel h5
template <typename R, int N>
__global__ void k_h6_pol(const R* h5p, const double* w, const R* h5ao, const double* wo, int P, cx<R>* h6) {
  constexpr long NR = long(N) * N * N;
  const long r = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= NR) return;
  double s = 0;
  for (int a = 0; a < P; ++a) s += w[a] * double(h5p[long(a) * NR + r]) + wo[a] * double(h5ao[long(a) * NR + r]);
  h6[r] = mk<R>(R(s), R(0));
}

// the same with the complex h5 of the biorthogonal mode
template <typename R, int N>
__global__ void k_h6_pol_c(const cx<R>* h5p, const double* w, const cx<R>* h5ao, const double* wo, int P,
                           cx<R>* h6) {
  constexpr long NR = long(N) * N * N;
  const long r = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= NR) return;
  double sr = 0, si = 0;
  for (int a = 0; a < P; ++a) {
    const cx<R> u = h5p[long(a) * NR + r], v = h5ao[long(a) * NR + r];
    sr += w[a] * double(u.x) + wo[a] * double(v.x);
    si += w[a] * double(u.y) + wo[a] * double(v.y);
  }
  h6[r] = mk<R>(R(sr), R(si));
}

// ---------------------------------------------------------------- pair passes
// Lattice components of the vector kernel.  With kappa_d = m_d + delta_d (grid frequency plus the
// pair's shift Delta, both in units of the reciprocal rows b_d), Q_c = sum_d kappa_d B_dc.  The
// Cartesian fields i Q_c u~ rho~ are therefore sum_d B_dc Y_d with Y_d = i kappa_d u~ rho~.  Along a
// z column kappa_1 and kappa_2 are constant, so the z stage needs two fields per spin channel,
// W0 = u~ rho~ and W3 = i kappa_3 u~ rho~, and the xy stage forms Y_1 = i kappa_1 W0,
// Y_2 = i kappa_2 W0, Y_3 = W3 before its inverse transform.  Forward contractions
// sum_c Q_c S~_c = sum_d kappa_d T~_d (T_d = sum_c B_dc S_c) are split the same way: the xy stage
// emits P = kappa_1 T~_1 + kappa_2 T~_2 and R = T~_3 and the z stage adds kappa_3 R~ to P~.
// Every plane kernel below uses one work-group per (target, z-plane, chunk of partners).

enum { OP_A1 = 0, OP_O = 1, OP_A2 = 2, OP_B = 3 };

struct Tables {
  const void* V;      // V2a (parallel), exchange conventions, [nDelta][N^3]
  const void* U1;     // u~ parallel
  const void* U2;     // u~ antiparallel
  const double* dfr;  // [nDelta][3] fractions of Delta
};

struct Masks {
  double m2ah, m2bh1, m2bh2, m2ax, m2bx1, m2bx2, m3a1, m3a2, m3a3, m3a4, m3b1, m3b2, m3b3, m3b4, m3b5, m3b6;
};

struct FusedArgs {
  int P, T, t0, S, chunk;     // orbitals, targets in batch, first target, partner chunks, partners per chunk
};

// The resident pair store of TC mode is triangular: row t holds the pass-A pairs (t, q) with q <= t and
// q < Q1, min(t + 1, Q1) of them, rows one after another.  The pair (t, q) of q > t is read from the pair
// (q, t): its density is the conjugate of (t, q)'s and its shift the negative, and every kernel that
// multiplies it is real in real space and zero on the Nyquist planes, so its z-stage output is the
// conjugate of (q, t)'s at the reflected frequencies, and every field that the plane kernels form from it
// (with its own shift) and transform to real space is the conjugate of (q, t)'s.  The plane kernels load
// (q, t) as it is, transform it with (q, t)'s shift and conjugate in real space.  Offset (in pairs) of row t:
__host__ __device__ __forceinline__ long tri_row(int t, int Q1) {
  return t < Q1 ? long(t) * (t + 1) / 2 : long(Q1) * (Q1 + 1) / 2 + long(t - Q1) * Q1;
}

// Pair p of a z-stage launch -> its row t of the batch and partner q.  Rectangular batches have rows of mi.P
// pairs.  A triangular one (mi.trq > 0) is the rows t0 + t of the triangular store with Q1 = trq, of
// min(t0 + t + 1, trq) pairs each, one after another; its input rows (the batch's pair planes) hold mi.P.
__host__ __device__ __forceinline__ void pair_tq(const MeshInfo& mi, int t0, long p, int& t, int& q) {
  if (mi.trq <= 0) {
    t = int(p / mi.P);
    q = int(p - long(t) * mi.P);
    return;
  }
  const long Q = mi.trq, g = tri_row(t0, mi.trq) + p, full = Q * (Q + 1) / 2;
  long r;
  if (g < full) {   // row r holds the pairs r (r + 1) / 2 .. (r + 1) (r + 2) / 2 - 1
    r = long((sqrt(8.0 * double(g) + 1.0) - 1.0) * 0.5);
    while (r * (r + 1) / 2 > g) --r;
    while ((r + 1) * (r + 2) / 2 <= g) ++r;
    q = int(g - r * (r + 1) / 2);
  } else {
    r = Q + (g - full) / Q;
    q = int(g - full - (r - Q) * Q);
  }
  t = int(r) - t0;
}

// index of the pair's shift in the kernel tables: k_jt - k_q (sign 1, target passes) or k_q - k_jt (sign 0);
// target jt sits at k-point jt / nbt, partner q at q / nb
__device__ __forceinline__ int pair_dindex(const MeshInfo& mi, int jt, int q, int sign) {
  const int kt = mi.tk ? mi.tk[jt / mi.nbt] : jt / mi.nbt, kq = (q + mi.qoff) / mi.nb;
  const int nkm = mi.n1 * mi.n2 * mi.n3;
  if (kt >= nkm) {   // band k-point: its own tables after the mesh differences, Delta = k_b - k_q then k_q - k_b
    const int nd = (2 * mi.n1 - 1) * (2 * mi.n2 - 1) * (2 * mi.n3 - 1);
    return nd + (sign ? 0 : mi.nkb * nkm) + (kt - nkm) * nkm + kq;
  }
  return sign ? kindex_delta(mi, kt, kq) : kindex_delta(mi, kq, kt);
}

template <typename R>
struct Basis {   // B_dc = component c of reciprocal row b_d, working precision
  R b[9];
};
template <typename R>
__device__ __forceinline__ Basis<R> basis(const Recip& rc) {
  Basis<R> B;
#pragma unroll
  for (int i = 0; i < 9; ++i) B.b[i] = R(rc.b[i]);
  return B;
}
// X_c = sum_d B_dc Y_d
template <typename R>
__device__ __forceinline__ void to_cart(const Basis<R>& B, const cx<R>* Y, cx<R>* X) {
#pragma unroll
  for (int c = 0; c < 3; ++c) X[c] = B.b[c] * Y[0] + B.b[3 + c] * Y[1] + B.b[6 + c] * Y[2];
}
// T_d = sum_c B_dc S_c
template <typename R>
__device__ __forceinline__ void to_latt(const Basis<R>& B, const cx<R>* S, cx<R>* T) {
#pragma unroll
  for (int d = 0; d < 3; ++d) T[d] = B.b[3 * d] * S[0] + B.b[3 * d + 1] * S[1] + B.b[3 * d + 2] * S[2];
}


// Lattice components of vector fields: out_d = sum_c B_dc in_c for nvec vectors of N^3 points;
// component c of vector v at in + v vstride + c cstride (same layout for out).
template <typename R, int N>
__global__ void k_lattice3(const cx<R>* in, cx<R>* out, Basis<R> B, long nvec, long vstride, long cstride) {
  constexpr long NR = long(N) * N * N;
  const long id = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id >= nvec * NR) return;
  const long v = id / NR, r = id - v * NR;
  const long o = v * vstride + r;
  cx<R> X[3], T[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) X[c] = in[o + c * cstride];
  to_latt(B, X, T);
#pragma unroll
  for (int d = 0; d < 3; ++d) out[o + d * cstride] = T[d];
}

template <typename R>
__device__ __forceinline__ void cfma(cx<R>& acc, R a, cx<R> u, cx<R> v) {   // acc += a u v
  const cx<R> p = u * v;
  acc.x += a * p.x;
  acc.y += a * p.y;
}

// Work-group layout of the plane kernels: RB rows x N columns of threads; thread (y0, x) owns the
// plane points (y0 + RB i, x), i < N/RB, so loads and stores are coalesced along x and need no index
// division.  Transforms of N <= 32 give each thread one line of one plane per pass (up to RB planes per
// pass); at N = 48 (COMB) the lines are split into their 3 x 16 prime-factor combs (planes_comb48).
template <typename R, int N>
struct Fz {
  // 48 points: 16 rows (768 threads, 12 waves on the one work-group that the LDS planes leave room for
  // per CU, 3 owned points per thread)
  static constexpr int RB = N == 48 ? 16 : (N % 8 == 0) ? 8 : 4;
  static constexpr int NTH = RB * N;
  static constexpr int KP = N / RB;
  static constexpr int LD = N + 1;
  static constexpr int PLANE = N * LD;                     // LDS elements per plane
  static constexpr int kLdsMax = 160 * 1024;               // LDS per work-group on gfx950
  static constexpr bool fits(int planes) { return planes * PLANE * int(sizeof(cx<R>)) <= kLdsMax; }
  static constexpr int kFitPlanes = kLdsMax / (PLANE * int(sizeof(cx<R>)));
  static constexpr int GRP = kFitPlanes < RB ? kFitPlanes : RB;   // one-plane-per-partner rounds
  // k_pair_xy and k_fused_Y (one plane per partner, few registers): in FP32 at 48 points 4 planes per round
  // (75 KB of LDS) at up to 6 waves per SIMD, so that two work-groups share a CU and overlap their phases
  static constexpr bool TWO_WG = sizeof(R) == 4 && N == 48;
  static constexpr int GRP1 = TWO_WG ? 4 : GRP;
  static constexpr int WAVES1 = TWO_WG ? 6 : 1;
  static constexpr bool COMB = N == 48;                    // comb transforms, outputs in sigma order
  // the next partner's planes are loaded into registers while this partner's are transformed; at 48
  // points the register budget allows it in FP32 only, and k_fused_A measured faster without it there
  static constexpr bool PREFETCH = N < 48 || sizeof(R) == 4;
  static constexpr bool PREFETCH_A = N < 48;
};

// Position of index k after the in-place comb transform of a 48-point axis (planes_comb48): the
// Good-Thomas map stores sub-index (k1, k2) = (k mod 3, k mod 16) at 16 k1 + 3 k2 (mod 48).
__device__ __forceinline__ int sigma48(int k) {
  const int r = 16 * (k % 3) + 3 * (k & 15);
  return r >= 48 ? r - 48 : r;
}

// One 16-point comb n1 of a 48-point line in LDS (element stride ST), transformed in place.
template <typename R, int DIR, int N1, int ST>
__device__ __forceinline__ void comb16(cx<R>* line) {
  cx<R> v[16];
#pragma unroll
  for (int n2 = 0; n2 < 16; ++n2) v[n2] = line[((16 * N1 + 3 * n2) % 48) * ST];
  fft_pow2<R, 16, DIR>(v);
#pragma unroll
  for (int n2 = 0; n2 < 16; ++n2) line[((16 * N1 + 3 * n2) % 48) * ST] = v[n2];
}

// The combs of np planes' lines along one axis, one (line, comb) per task: every thread of the
// work-group takes part.  The comb index is uniform over most waves; it selects one of three
// compile-time address patterns.
template <typename R, int DIR, bool COL, bool FENCE = false>
__device__ __forceinline__ void comb_pass48(cx<R>* sm, int np, int tid, int nth) {
  constexpr int N = 48, LD = N + 1, PL = N * LD;
  const int nl = np * N;
  for (int t = tid; t < 3 * nl; t += nth) {
    int tt = t;   // FENCE: recomputed per pass, not held across the caller's loop (compiler-only fence)
    if constexpr (FENCE) asm volatile("" : "+v"(tt));
    const int n1 = tt / nl, r = tt - n1 * nl;
    const int p = r / N, l = r - p * N;
    cx<R>* line = COL ? sm + p * PL + l : sm + p * PL + l * LD;
    if (n1 == 0)
      comb16<R, DIR, 0, COL ? LD : 1>(line);
    else if (n1 == 1)
      comb16<R, DIR, 1, COL ? LD : 1>(line);
    else
      comb16<R, DIR, 2, COL ? LD : 1>(line);
  }
  __syncthreads();
}

// In-place 2D transform of np 48 x 48 planes in LDS ([np][48][49]) in three passes over the
// prime-factor (Good-Thomas) structure 48 = 3 x 16, which has no twiddles between its factors:
//   1. every row: the three 16-point transforms over n2 of its combs n1 (positions 16 n1 + 3 n2 mod 48);
//   2. every column: the same along y;
//   3. every (k2x, k2y): the 3 x 3 transform over (n1x, n1y).
// Each pass writes back to the positions it read, so sub-index (a, b) stays at 16 a + 3 b (mod 48).
// With the input index in natural order (the Ruritanian map n = 16 n1 + 3 n2) the output index is the
// Chinese-remainder map k = 16 k1 + 33 k2, so output k sits at sigma48(k) on each axis; with the input
// at sigma48 positions the output is in natural order (the two maps swap roles).  A thread holds one
// 16-point comb (32 registers in FP32) instead of a 48-point line.  Ends with a barrier.
// BAL: the row and column passes take one (line, comb) per task (comb_pass48); otherwise the row pass gives
// a thread a whole row's three combs in turn (fewer threads busy, a shorter instruction stream) and the
// column pass takes one (column, comb) per task, which measured faster in k_fused_A's inverse transforms
// and slower everywhere else (k_fused_A's forward transforms, k_fused_O, k_passB_xy, k_fused_Y, k_pair_xy).
// FENCE: the task addresses are recomputed in each call rather than kept in registers across the caller's
// loop (for a kernel whose registers are short).
template <typename R, int DIR, bool BAL, bool FENCE = false>
__device__ __forceinline__ void planes_comb48(cx<R>* sm, int np, int tid, int nth) {
  constexpr int N = 48, LD = N + 1, PL = N * LD;
  if constexpr (BAL) {
    comb_pass48<R, DIR, false, FENCE>(sm, np, tid, nth);
    comb_pass48<R, DIR, true, FENCE>(sm, np, tid, nth);
  } else {
    for (int t = tid; t < np * N; t += nth) {
      const int p = t / N, y = t - p * N;
      cx<R>* row = sm + p * PL + y * LD;
      comb16<R, DIR, 0, 1>(row);
      __builtin_amdgcn_sched_barrier(0);   // one comb in registers at a time
      comb16<R, DIR, 1, 1>(row);
      __builtin_amdgcn_sched_barrier(0);
      comb16<R, DIR, 2, 1>(row);
    }
    __syncthreads();
    comb_pass48<R, DIR, true, FENCE>(sm, np, tid, nth);
  }
  for (int t = tid; t < np * 256; t += nth) {
    int tt = t;
    if constexpr (FENCE) asm volatile("" : "+v"(tt));
    const int p = tt >> 8, ky = (tt >> 4) & 15, kx = tt & 15;
    cx<R>* pl = sm + p * PL;
    int xo[3], yo[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const int xa = 16 * a + 3 * kx, ya = 16 * a + 3 * ky;
      xo[a] = xa >= N ? xa - N : xa;
      yo[a] = (ya >= N ? ya - N : ya) * LD;
    }
    cx<R> v[3][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) v[a][b] = pl[yo[a] + xo[b]];
#pragma unroll
    for (int a = 0; a < 3; ++a) dft3<R, DIR>(v[a]);
#pragma unroll
    for (int b = 0; b < 3; ++b) {
      cx<R> c[3] = {v[0][b], v[1][b], v[2][b]};
      dft3<R, DIR>(c);
#pragma unroll
      for (int a = 0; a < 3; ++a) v[a][b] = c[a];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) pl[yo[a] + xo[b]] = v[a][b];
  }
  __syncthreads();
}

// in-place 2D transform of np planes in LDS ([np][N][N+1]); thread row p takes planes p, p + RB, ...;
// ends with a barrier.  The plane kernels below write and read LDS outside these transforms only at the
// points each thread owns (PlaneWG::so, natural order), so a round's reads after a transform and the next
// round's writes need no barrier between them: only the barrier before the next transform.  At N = 48
// the transform is planes_comb48: reads after it use PlaneWG::ss (sigma order), and a barrier separates
// them from the next round's writes (end_round).
template <typename R, int N, int DIR, bool BAL = false, bool FENCE = false>
__device__ __forceinline__ void planes_fft(cx<R>* sm, int np, int tid) {
  if constexpr (Fz<R, N>::COMB) {
    planes_comb48<R, DIR, BAL, FENCE>(sm, np, tid, Fz<R, N>::NTH);
    return;
  }
  constexpr int LD = N + 1, RB = Fz<R, N>::RB;
  const int p0 = tid / N, l = tid - (tid / N) * N;
  for (int p = p0; p < np; p += RB) {
    cx<R> v[N];
    cx<R>* row = sm + (p * N + l) * LD;
#pragma unroll
    for (int x = 0; x < N; ++x) v[x] = row[x];
    fft_line<R, N, DIR>(v);
#pragma unroll
    for (int x = 0; x < N; ++x) row[x] = v[x];
  }
  __syncthreads();
  for (int p = p0; p < np; p += RB) {
    cx<R> v[N];
    cx<R>* col = sm + p * N * LD + l;
#pragma unroll
    for (int y = 0; y < N; ++y) v[y] = col[y * LD];
    fft_line<R, N, DIR>(v);
#pragma unroll
    for (int y = 0; y < N; ++y) col[y * LD] = v[y];
  }
  __syncthreads();
}

// Access base[byte offset] with a work-group-uniform base and a 32-bit lane offset, so that the
// compiler can use the scalar-base + 32-bit vector-offset addressing form.
template <typename T>
__device__ __forceinline__ T ldo(const T* base, unsigned byteoff) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(base) + byteoff);
}
template <typename T>
__device__ __forceinline__ void sto(T* base, unsigned byteoff, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(base) + byteoff) = v;
}
// A work-group-uniform global pointer, read from the first lane and typed as global memory, so that the
// loads through it take the scalar-base + 32-bit vector-offset form with no per-lane address arithmetic.
template <typename T>
using gptr = const __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> uniform_global(const T* p) {
  const unsigned long long v = reinterpret_cast<unsigned long long>(p);
  const unsigned lo = __builtin_amdgcn_readfirstlane(unsigned(v));
  const unsigned hi = __builtin_amdgcn_readfirstlane(unsigned(v >> 32));
  return reinterpret_cast<gptr<T>>((static_cast<unsigned long long>(hi) << 32) | lo);
}
// A value at a wave-uniform address of a table that no kernel writes, read with a scalar load (into
// scalar registers, without waiting on the vector memory counter)
template <typename T>
__device__ __forceinline__ T ld_uniform(const T* p) {
  const unsigned long long v = reinterpret_cast<unsigned long long>(p);
  const unsigned lo = __builtin_amdgcn_readfirstlane(unsigned(v));
  const unsigned hi = __builtin_amdgcn_readfirstlane(unsigned(v >> 32));
  return *reinterpret_cast<const __attribute__((address_space(4))) T*>((static_cast<unsigned long long>(hi) << 32) | lo);
}
template <typename R>
__device__ __forceinline__ cx<R> ldo(gptr<cx<R>> base, unsigned byteoff) {
  typedef R v2 __attribute__((ext_vector_type(2)));
  const v2 v = *reinterpret_cast<const __attribute__((address_space(1))) v2*>(
      reinterpret_cast<const __attribute__((address_space(1))) char*>(base) + byteoff);
  return mk<R>(v.x, v.y);
}

// Logical work-group index from the hardware one.  Work-groups are dealt to the 8 XCDs round-robin;
// this map gives each XCD a contiguous range of logical indices (bijective for any grid size).
__device__ __forceinline__ int xcd_major(int b, int n) {
  const int q8 = n / 8, r8 = n % 8, x = b % 8;
  return x * q8 + min(x, r8) + b / 8;
}

// common decoding of a plane-kernel work-group: logical index = (z-plane, chunk) major, target minor,
// so the work-groups of all targets that read the same partner planes run together on one XCD and
// share its L2
template <typename R, int N>
struct PlaneWG {
  using F = Fz<R, N>;
  int x, y0, c, z, t, qb, qe;
  unsigned zo;   // offset of owned point i within a volume: zo + RB N i
  int so0;       // LDS offset of owned point i: so0 + RB LD i
  int sx;        // column of owned points after a comb transform (sigma48(x); N = 48 only)
  __device__ PlaneWG(const FusedArgs& fa) {
    const int tid = threadIdx.x;
    x = tid % N;
    y0 = tid / N;
    const int L = xcd_major(int(blockIdx.x), int(gridDim.x));
    t = L % fa.T;
    c = (L / fa.T) % fa.S;
    z = L / (fa.T * fa.S);
    qb = c * fa.chunk;
    qe = min(fa.P, qb + fa.chunk);
    zo = unsigned(z * N * N + y0 * N + x);
    so0 = y0 * F::LD + x;
    sx = F::COMB ? sigma48(x) : x;
  }
  // LDS offset of owned point i in natural order (inputs of a transform; outputs of one whose input was
  // in sigma order)
  __device__ __forceinline__ int so(int i) const { return so0 + F::RB * F::LD * i; }
  // LDS offset of owned point i after a transform of natural-order input (sigma order at N = 48)
  __device__ __forceinline__ int ss(int i) const {
    if constexpr (F::COMB)
      return sigma48(y0 + F::RB * i) * F::LD + sx;
    else
      return so(i);
  }
  // between a round's reads at ss() and the next round's writes at so(): a barrier where they differ
  __device__ __forceinline__ void end_round() const {
    if constexpr (F::COMB) __syncthreads();
  }
};

// Pair densities rho = conj(bra_a) ket_b, forward xy transformed, for the pairs (t, q) of a target
// batch: TFIRST a = t0 + t, b = q; else a = q, b = t0 + t.  out[(t P + q)][N^3].  bra holds the left
// orbitals chi (the right ones, psi, in TC mode), ket the right ones.
template <typename R, int N, bool TFIRST>
__global__ void __launch_bounds__((Fz<R, N>::NTH)) __attribute__((amdgpu_waves_per_eu(Fz<R, N>::WAVES1)))
k_pair_xy(const cx<R>* bra, const cx<R>* ket, FusedArgs fa,
                                                           cx<R>* out) {
  using F = Fz<R, N>;
  constexpr int KP = F::KP, RB = F::RB;
  constexpr long NR = long(N) * N * N;
  __shared__ cx<R> sm[F::GRP1 * F::PLANE];
  const PlaneWG<R, N> wg(fa);
  const cx<R>* tf = TFIRST ? bra : ket;   // field of the target index
  const cx<R>* pf = TFIRST ? ket : bra;   // field of the partner index
  cx<R> pt[KP];
#pragma unroll
  for (int i = 0; i < KP; ++i) pt[i] = tf[long(fa.t0 + wg.t) * NR + wg.zo + RB * N * i];
  for (int q0 = wg.qb; q0 < wg.qe; q0 += F::GRP1) {
    const int nq = min(F::GRP1, wg.qe - q0);
    for (int cc = 0; cc < nq; ++cc) {
      const cx<R>* pq = pf + long(q0 + cc) * NR + wg.zo;
#pragma unroll
      for (int i = 0; i < KP; ++i)
        sm[cc * F::PLANE + wg.so0 + RB * F::LD * i] = TFIRST ? cmulc(pt[i], pq[RB * N * i]) : cmulc(pq[RB * N * i], pt[i]);
    }
    __syncthreads();
    planes_fft<R, N, -1, true>(sm, nq, threadIdx.x);
    for (int cc = 0; cc < nq; ++cc) {
      cx<R>* dst = out + (long(wg.t) * fa.P + q0 + cc) * NR + wg.zo;
#pragma unroll
      for (int i = 0; i < KP; ++i) dst[RB * N * i] = sm[cc * F::PLANE + wg.ss(i)];
    }
    wg.end_round();
  }
}

// Pass-B sources of the pairs (t, q), in lattice components: T_d = conj(chi_q) Zl_td +
// m3b5 conj(Hl_qd) psi_t, with Zl = B (m2bx2 D_j - m3b3 h1 psi_j + m3b4 h4_j) and Hl = B conj(H3b)
// (TC mode: chi = psi and H3b = conj(H3a4), so Hl = B H3a4); forward xy transformed:
// out[(pair 2 + 0)] = kappa_1 T~_1 + kappa_2 T~_2, out[(pair 2 + 1)] = T~_3, pair = t P + q, Delta = k_t - k_q.
// FP32 at 24^3: no register prefetch of the partner fields, 4 waves per SIMD instead (no spills); FP64 at 48
// points none either (register budget); elsewhere the prefetch
template <typename R, int N>
constexpr bool kPassBPrefetch = !(sizeof(R) == 4 && N == 24) && Fz<R, N>::PREFETCH;
template <typename R, int N>
constexpr int kPassBWaves = (sizeof(R) == 4 && N == 24) ? 4 : 1;

template <typename R, int N>
__global__ void __launch_bounds__((Fz<R, N>::NTH)) __attribute__((amdgpu_waves_per_eu(kPassBWaves<R, N>)))
k_passB_xy(const cx<R>* psi, const cx<R>* chi, const cx<R>* Zl, const cx<R>* Hl, FusedArgs fa, MeshInfo mi,
           const double* dfr, R m3b5, cx<R>* out) {
  using F = Fz<R, N>;
  constexpr int KP = F::KP, RB = F::RB;
  constexpr int NPQ = F::GRP / 3 < 1 ? 1 : F::GRP / 3;   // partners per LDS round (three planes each)
  constexpr long NR = long(N) * N * N;
  __shared__ cx<R> sm[3 * NPQ * F::PLANE];
  const PlaneWG<R, N> wg(fa);
  const long jt = fa.t0 + wg.t;
  cx<R> zt[KP][3], pt[KP];
  {
    const cx<R>* pj = psi + jt * NR;
    const cx<R>* zb = Zl + long(wg.t) * 3 * NR;
#pragma unroll
    for (int i = 0; i < KP; ++i) {
      const unsigned r = wg.zo + RB * N * i;
      pt[i] = pj[r];
#pragma unroll
      for (int d = 0; d < 3; ++d) zt[i][d] = zb[d * NR + r];
    }
  }
  // partner fields chi_q, Hl_q of the next round are loaded while this round is transformed (kPassBPrefetch;
  // otherwise at the start of the round)
  constexpr bool PF = kPassBPrefetch<R, N>;
  cx<R> pre[NPQ][4][KP];
  auto fetch = [&](int q0) {
#pragma unroll
    for (int a = 0; a < NPQ; ++a) {
      const int q = min(q0 + a, wg.qe - 1);
      const cx<R>* pq = chi + long(q) * NR;
      const cx<R>* hq = Hl + long(q) * 3 * NR;
#pragma unroll
      for (int i = 0; i < KP; ++i) {
        const unsigned r = wg.zo + RB * N * i;
        pre[a][0][i] = pq[r];
#pragma unroll
        for (int d = 0; d < 3; ++d) pre[a][1 + d][i] = hq[d * NR + r];
      }
    }
  };
  if (PF && wg.qb < wg.qe) fetch(wg.qb);
  for (int q0 = wg.qb; q0 < wg.qe; q0 += NPQ) {
    const int nq = min(NPQ, wg.qe - q0);
    if (!PF) fetch(q0);
#pragma unroll
    for (int a = 0; a < NPQ; ++a) {
      if (a >= nq) continue;
#pragma unroll
      for (int i = 0; i < KP; ++i) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          cx<R> T = cmulc(pre[a][0][i], zt[i][d]);
          if (m3b5 != R(0)) T = T + m3b5 * cmulc(pre[a][1 + d][i], pt[i]);
          sm[(3 * a + d) * F::PLANE + wg.so0 + RB * F::LD * i] = T;
        }
      }
    }
    if (PF && q0 + NPQ < wg.qe) fetch(q0 + NPQ);
    __syncthreads();
    planes_fft<R, N, -1, true>(sm, 3 * nq, threadIdx.x);
    for (int a = 0; a < nq; ++a) {
      const int q = q0 + a;
      const double* dl = dfr + 3 * pair_dindex(mi, int(jt), q, 1);
      const double del[2] = {ld_uniform(dl), ld_uniform(dl + 1)};
      const R k1 = R(double(mfreq<N>(wg.x)) + del[0]);
      cx<R>* dst = out + (long(wg.t) * fa.P + q) * 2 * NR;
#pragma unroll
      for (int i = 0; i < KP; ++i) {
        const int so = (3 * a) * F::PLANE + wg.ss(i);
        const unsigned r = wg.zo + RB * N * i;
        const R k2 = R(double(mfreq<N>(wg.y0 + RB * i)) + del[1]);
        dst[r] = k1 * sm[so] + k2 * sm[so + F::PLANE];
        dst[NR + r] = sm[so + 2 * F::PLANE];
      }
    }
    wg.end_round();
  }
}

// z stage of a pair convolution: forward z transform of the inputs, kernel multiply at Q = Delta + G
// for the pair's Delta, inverse z transform of each output (one thread per (pair, x, y) column).
//   OP_O : 1 -> 4  [W0_par, W3_par, W0_anti, W3_anti]
//   OP_A1: 1 -> 5  [V2a_par rho, W0_par, W3_par, W0_anti, W3_anti]
//          W0_s = u~_s rho, W3_s = i kappa_3 u~_s rho
//   OP_A2: 4 -> 1  -i sum_s u~_s (P_s + kappa_3 R_s), inputs [P_par, R_par, P_anti, R_anti]
//   OP_B : 2 -> 1  +i u~_par (P + kappa_3 R), inputs [P, R]
// OP_A2 with inB ([pair][2] pass-B sources [P_B, R_B]): -u~_par (P_B + kappa_3 R_B) joins the sum, so that
// the one output is the sum of the OP_A2 and OP_B outputs (both take u~_par).
template <int OP>
struct OpShape;
template <> struct OpShape<OP_A1> { static constexpr int nin = 1, nout = 5; };
template <> struct OpShape<OP_O> { static constexpr int nin = 1, nout = 4; };
template <> struct OpShape<OP_A2> { static constexpr int nin = 4, nout = 1; };
template <> struct OpShape<OP_B> { static constexpr int nin = 2, nout = 1; };

// occupancy target: 3 waves per SIMD for FP32 at 24^3 (every operation fits 168 registers there)
template <typename R, int N>
constexpr int kZconvWaves = (sizeof(R) == 4 && N == 24) ? 3 : 1;

template <typename R, int N, int OP>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kZconvWaves<R, N>)))
k_zconv(const cx<R>* in, cx<R>* out, long npairs, int t0, MeshInfo mi, Tables tb, int sign_target_minus_partner,
        const cx<R>* inB = nullptr) {
  constexpr int NN = N * N;
  constexpr long NR = long(N) * N * N;
  constexpr int NIN = OpShape<OP>::nin, NOUT = OpShape<OP>::nout;
  const long col = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (col >= npairs * NN) return;
  const long pair = col / NN;
  const int xy = int(col - pair * NN);
  int t, q;
  pair_tq(mi, t0, pair, t, q);
  const int di = pair_dindex(mi, t0 + t, q, sign_target_minus_partner);
  const R* tV = reinterpret_cast<const R*>(tb.V) + long(di) * NR + xy;
  const R* tU[2] = {reinterpret_cast<const R*>(tb.U1) + long(di) * NR + xy,
                    reinterpret_cast<const R*>(tb.U2) + long(di) * NR + xy};
  const R d3 = R(tb.dfr[3 * di + 2]);   // kappa_3(z) = m_z + delta_3

  if constexpr (NIN == 1) {
    cx<R> acc[N], v[N];
    const cx<R>* b = in + (long(t) * mi.P + q) * NR + xy;
#pragma unroll
    for (int z = 0; z < N; ++z) acc[z] = b[z * NN];
    fft_line<R, N, -1>(acc);
    cx<R>* o = out + pair * NOUT * NR + xy;
    if constexpr (OP == OP_A1) {
#pragma unroll
      for (int z = 0; z < N; ++z) v[z] = tV[z * NN] * acc[z];
      fft_line<R, N, 1>(v);
#pragma unroll
      for (int z = 0; z < N; ++z) o[z * NN] = v[z];
      o += NR;
    }
#pragma unroll 1
    for (int s = 0; s < 2; ++s) {
      R u[N];
#pragma unroll
      for (int z = 0; z < N; ++z) u[z] = tU[s][z * NN];
#pragma unroll
      for (int z = 0; z < N; ++z) v[z] = u[z] * acc[z];
      fft_line<R, N, 1>(v);
#pragma unroll
      for (int z = 0; z < N; ++z) o[z * NN] = v[z];
#pragma unroll
      for (int z = 0; z < N; ++z) v[z] = mul_i(((R(mfreq<N>(z)) + d3) * u[z]) * acc[z]);
      fft_line<R, N, 1>(v);
#pragma unroll
      for (int z = 0; z < N; ++z) o[NR + z * NN] = v[z];
      o += 2 * NR;
    }
  } else {
    cx<R> acc[N], v[N];
#pragma unroll
    for (int z = 0; z < N; ++z) acc[z] = mk<R>(R(0), R(0));
    // channels: the NIN / 2 input pairs, then (OP_A2 with inB) the pass-B sources with u~_par and sign -1
    const int nch = NIN / 2 + ((OP == OP_A2 && inB) ? 1 : 0);
#pragma unroll 1
    for (int s = 0; s < nch; ++s) {
      const bool isB = s == NIN / 2;
      const cx<R>* b = isB ? inB + pair * 2 * NR + xy : in + (pair * NIN + 2 * s) * NR + xy;
      const R* tu = (s == 1 && !isB) ? tU[1] : tU[0];
      const R sg = isB ? R(-1) : R(1);
#pragma unroll
      for (int z = 0; z < N; ++z) v[z] = b[z * NN];
      fft_line<R, N, -1>(v);
#pragma unroll
      for (int z = 0; z < N; ++z) acc[z] = acc[z] + (sg * tu[z * NN]) * v[z];
#pragma unroll
      for (int z = 0; z < N; ++z) v[z] = b[NR + z * NN];
      fft_line<R, N, -1>(v);
#pragma unroll
      for (int z = 0; z < N; ++z) acc[z] = acc[z] + ((R(mfreq<N>(z)) + d3) * (sg * tu[z * NN])) * v[z];
    }
#pragma unroll
    for (int z = 0; z < N; ++z) acc[z] = OP == OP_A2 ? mul_i(R(-1) * acc[z]) : mul_i(acc[z]);
    fft_line<R, N, 1>(acc);
    cx<R>* o = out + pair * NR + xy;
#pragma unroll
    for (int z = 0; z < N; ++z) o[z * NN] = acc[z];
  }
}

// ---------------------------------------------------------------- 48-point z stage on lane pairs
// A 48-point column split over two adjacent lanes (h = lane & 1): radix 2 by decimation in frequency, then
// the 24-point prime-factor transform in registers.  Lane h holds z = 24 h + j (j < 24) in real space and
// frequency k = 2 j + h after the forward half.  The butterfly partner of each value is in lane ^ 1,
// read with a DPP quad permutation (no LDS, no barrier).  One thread then holds 24 values per field
// instead of 48, which keeps the z stage at 3 waves per SIMD.
template <typename R>
__device__ __forceinline__ R lane_swap(R v) {   // the value of lane ^ 1
  if constexpr (sizeof(R) == 4) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, false));
  } else {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_mov_dpp(int(b), 0xB1, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(int(b >> 32), 0xB1, 0xF, 0xF, false);
    return __longlong_as_double((static_cast<long long>(hi) << 32) | static_cast<unsigned>(lo));
  }
}
template <typename R>
__device__ __forceinline__ cx<R> lane_swap(cx<R> v) { return mk<R>(lane_swap(v.x), lane_swap(v.y)); }

// r e^{DIR 2 pi i j / 48} on lanes h = 1 (hf = 1), r on lanes h = 0 (hf = 0): r + hf (r w - r), with the
// twiddle w read from the constant table (uniform), so that no per-lane twiddle is kept in registers
template <typename R, int DIR>
__device__ __forceinline__ cx<R> half_twiddle_mul(cx<R> r, int j, R hf) {
  const cx<R> w = twiddle<R, 48, DIR>(j);
  const cx<R> d = mk<R>(r.x * w.x - r.y * w.y - r.x, r.x * w.y + r.y * w.x - r.y);
  return mk<R>(r.x + hf * d.x, r.y + hf * d.y);
}

// forward: x[24 h + j] -> X[2 j + h]; hf = h (0 or 1)
template <typename R>
__device__ __forceinline__ void fwd48_pair(cx<R>* v, R hf) {
  const R s = R(1) - R(2) * hf;
#pragma unroll
  for (int j = 0; j < 24; ++j) {
    const cx<R> o = lane_swap(v[j]);
    const cx<R> r = mk<R>(o.x + s * v[j].x, o.y + s * v[j].y);   // h = 0: x_j + x_j+24; h = 1: x_j - x_j+24
    v[j] = j == 0 ? r : half_twiddle_mul<R, -1>(r, j, hf);
  }
  fft_line<R, 24, -1>(v);
}

// inverse (unnormalised): X[2 j + h] -> x[24 h + j]
template <typename R>
__device__ __forceinline__ void inv48_pair(cx<R>* v, R hf) {
  fft_line<R, 24, 1>(v);   // h = 0: even-frequency part e_j; h = 1: odd part o_j
  const R s = R(1) - R(2) * hf;
#pragma unroll
  for (int j = 0; j < 24; ++j) {
    const cx<R> t = j == 0 ? v[j] : half_twiddle_mul<R, 1>(v[j], j, hf);   // h = 1: e^{2 pi i j/48} o_j
    const cx<R> o = lane_swap(t);
    v[j] = mk<R>(o.x + s * t.x, o.y + s * t.y);   // h = 0: e_j + w o_j; h = 1: e_j - w o_j
  }
}

// The z stage of k_zconv at N = 48 with each column on a lane pair (same operations, inputs and outputs).
template <typename R, int OP>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 && OP != OP_A2 ? 3 : 2)))
k_zconv48(const cx<R>* in, cx<R>* out, long npairs, int t0, MeshInfo mi, Tables tb, int sign_target_minus_partner,
          const cx<R>* inB = nullptr) {
  constexpr int N = 48, H = 24, NN = N * N;
  constexpr long NR = long(N) * N * N;
  constexpr int NIN = OpShape<OP>::nin, NOUT = OpShape<OP>::nout;
  const long gid = long(blockIdx.x) * blockDim.x + threadIdx.x;
  const long col = gid >> 1;
  const bool h = (threadIdx.x & 1) != 0;
  const R hf = h ? R(1) : R(0);
  // both lanes of a pair run every instruction (the grid covers whole pairs: npairs * NN * 2 threads)
  if (col >= npairs * NN) return;
  const long pair = col / NN;
  const int xy = int(col - pair * NN);
  int t, q;
  pair_tq(mi, t0, pair, t, q);
  const int di = pair_dindex(mi, t0 + t, q, sign_target_minus_partner);
  // frequency of element j after the forward half: k = 2 j + h; real-space z = 24 h + j
  const long kof = long(di) * NR + xy + (h ? NN : 0);
  const R* tV = reinterpret_cast<const R*>(tb.V) + kof;
  const R* tU0 = reinterpret_cast<const R*>(tb.U1) + kof;
  const R* tU1 = reinterpret_cast<const R*>(tb.U2) + kof;
  // kappa_3 = m_z + delta_3 at frequency 2 j + h: m(2 j) + h + delta_3 (2 j and 2 j + 1 never straddle N/2)
  const R d3h = R(tb.dfr[3 * di + 2]) + hf;
  const int zo = h ? H * NN : 0;
  auto kap3 = [&](int j) { return R(mfreq<N>(2 * j)) + d3h; };

  if constexpr (NIN == 1) {
    cx<R> acc[H], v[H];
    const cx<R>* b = in + (long(t) * mi.P + q) * NR + xy + zo;
#pragma unroll
    for (int j = 0; j < H; ++j) acc[j] = b[j * NN];
    fwd48_pair(acc, hf);
    __builtin_amdgcn_sched_barrier(0);   // phases in order: one field's values in registers at a time
    cx<R>* o = out + pair * NOUT * NR + xy + zo;
    if constexpr (OP == OP_A1) {
#pragma unroll
      for (int j = 0; j < H; ++j) v[j] = tV[2 * j * NN] * acc[j];
      inv48_pair(v, hf);
#pragma unroll
      for (int j = 0; j < H; ++j) o[j * NN] = v[j];
      __builtin_amdgcn_sched_barrier(0);
      o += NR;
    }
#pragma unroll 1
    for (int s = 0; s < 2; ++s) {
      const R* tu = s ? tU1 : tU0;
#pragma unroll
      for (int j = 0; j < H; ++j) v[j] = tu[2 * j * NN] * acc[j];
      inv48_pair(v, hf);
#pragma unroll
      for (int j = 0; j < H; ++j) o[j * NN] = v[j];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int j = 0; j < H; ++j) v[j] = mul_i((kap3(j) * tu[2 * j * NN]) * acc[j]);
      inv48_pair(v, hf);
#pragma unroll
      for (int j = 0; j < H; ++j) o[NR + j * NN] = v[j];
      __builtin_amdgcn_sched_barrier(0);
      o += 2 * NR;
    }
  } else if constexpr (OP == OP_A2 && sizeof(R) == 4) {
    // software pipeline (FP32 at 2 waves per SIMD): the next input is requested before this one is
    // transformed; input k is channel k / 2, its P (even k) or R (odd k) field
    cx<R> acc[H], v[H], nx[H];
#pragma unroll
    for (int j = 0; j < H; ++j) acc[j] = mk<R>(R(0), R(0));
    const int nin = 2 * (NIN / 2 + (inB ? 1 : 0));
    auto src = [&](int k) -> const cx<R>* {
      const int s = k >> 1;
      return (s == NIN / 2 ? inB + pair * 2 * NR : in + (pair * NIN + 2 * s) * NR) + (k & 1) * NR + xy + zo;
    };
    {
      const cx<R>* b = src(0);
#pragma unroll
      for (int j = 0; j < H; ++j) v[j] = b[j * NN];
    }
#pragma unroll 1
    for (int k = 0; k < nin; ++k) {
      if (k + 1 < nin) {
        const cx<R>* b = src(k + 1);
#pragma unroll
        for (int j = 0; j < H; ++j) nx[j] = b[j * NN];
      }
      fwd48_pair(v, hf);
      const int s = k >> 1;
      const bool isB = s == NIN / 2;
      const R* tu = (s == 1 && !isB) ? tU1 : tU0;
      const R sg = isB ? R(-1) : R(1);
      if (k & 1) {
#pragma unroll
        for (int j = 0; j < H; ++j) acc[j] = acc[j] + (kap3(j) * (sg * tu[2 * j * NN])) * v[j];
      } else {
#pragma unroll
        for (int j = 0; j < H; ++j) acc[j] = acc[j] + (sg * tu[2 * j * NN]) * v[j];
      }
#pragma unroll
      for (int j = 0; j < H; ++j) v[j] = nx[j];
    }
#pragma unroll
    for (int j = 0; j < H; ++j) acc[j] = mul_i(R(-1) * acc[j]);
    inv48_pair(acc, hf);
    cx<R>* o = out + pair * NR + xy + zo;
#pragma unroll
    for (int j = 0; j < H; ++j) o[j * NN] = acc[j];
  } else {
    cx<R> acc[H], v[H];
#pragma unroll
    for (int j = 0; j < H; ++j) acc[j] = mk<R>(R(0), R(0));
    const int nch = NIN / 2 + ((OP == OP_A2 && inB) ? 1 : 0);
#pragma unroll 1
    for (int s = 0; s < nch; ++s) {
      const bool isB = s == NIN / 2;
      const cx<R>* b = (isB ? inB + pair * 2 * NR : in + (pair * NIN + 2 * s) * NR) + xy + zo;
      const R* tu = (s == 1 && !isB) ? tU1 : tU0;
      const R sg = isB ? R(-1) : R(1);
#pragma unroll
      for (int j = 0; j < H; ++j) v[j] = b[j * NN];
      fwd48_pair(v, hf);
#pragma unroll
      for (int j = 0; j < H; ++j) acc[j] = acc[j] + (sg * tu[2 * j * NN]) * v[j];
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int j = 0; j < H; ++j) v[j] = b[NR + j * NN];
      fwd48_pair(v, hf);
#pragma unroll
      for (int j = 0; j < H; ++j) acc[j] = acc[j] + (kap3(j) * (sg * tu[2 * j * NN])) * v[j];
      __builtin_amdgcn_sched_barrier(0);
    }
#pragma unroll
    for (int j = 0; j < H; ++j) acc[j] = OP == OP_A2 ? mul_i(R(-1) * acc[j]) : mul_i(acc[j]);
    inv48_pair(acc, hf);
    cx<R>* o = out + pair * NR + xy + zo;
#pragma unroll
    for (int j = 0; j < H; ++j) o[j * NN] = acc[j];
  }
}

// ---------------------------------------------------------------- z stage on the matrix cores
// Split-BF16 variant of k_zconv (working precision FP32): every length-N DFT along z is a dense real
// GEMM on v_mfma_f32_16x16x16_bf16.  A column of N complex values is a real vector of 2N rows with
// real and imaginary parts interleaved (row 2z + c), so the DFT is the 2N x 2N real matrix with 2x2
// blocks [[w_r, -w_i], [w_i, w_r]], w = e^{DIR 2 pi i z' z / N}, cut into NT x NT tiles of 16 x 16
// (NT = N/8).  A wave owns 16 columns.  Operand lane layouts (16x16x16): A lane l holds
// A[l%16][4(l/16) + j], B lane l holds B[4(l/16) + j][l%16], D lane l holds D[4(l/16) + v][l%16],
// j, v = 0..3; with interleaved rows a lane therefore holds two consecutive complex values
// (z = 8 tile + 2(l/16) + {0, 1}) of its column in A-, B- and D-form alike, and a DFT's result feeds
// the next DFT as its B operand unchanged.  Each operand x is split x = hi + lo in BF16
// (round-to-nearest-even, lo = bf16(x - hi)) and a product is hi_A hi_B + hi_A lo_B + lo_A hi_B,
// accumulated in FP32.  The matrix fragments (both directions, hi and lo) come from the host in lane
// order and are staged in LDS.
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int N>
struct ZMfma {
  static constexpr int NT = N / 8;                     // 16-row tiles of 2N interleaved rows
  static constexpr int NFRAG = 2 * 2 * NT * NT * 64;   // [dir][hi/lo][mt][kt][lane]
  static constexpr int frag(int dir, int hl, int mt, int kt) { return (((dir * 2 + hl) * NT + mt) * NT + kt) * 64; }
};

__device__ __forceinline__ unsigned bf16x2_rne(float a, float b) {
  __hip_bfloat162 p = __float22bfloat162_rn(make_float2(a, b));
  return *reinterpret_cast<unsigned*>(&p);     // low half a, high half b
}

// x (4 FP32 rows of one lane) -> hi, lo in BF16
__device__ __forceinline__ void split_bf16(const f32x4& x, bf16x4& hi, bf16x4& lo) {
  const unsigned h0 = bf16x2_rne(x.x, x.y), h1 = bf16x2_rne(x.z, x.w);
  const float r0 = x.x - __uint_as_float(h0 << 16), r1 = x.y - __uint_as_float(h0 & 0xffff0000u);
  const float r2 = x.z - __uint_as_float(h1 << 16), r3 = x.w - __uint_as_float(h1 & 0xffff0000u);
  const unsigned l0 = bf16x2_rne(r0, r1), l1 = bf16x2_rne(r2, r3);
  uint2 uh{h0, h1}, ul{l0, l1};
  hi = *reinterpret_cast<bf16x4*>(&uh);
  lo = *reinterpret_cast<bf16x4*>(&ul);
}

// A fragment of the DFT matrix, read through an LDS (address space 3) pointer so that it is a ds_read
typedef const __attribute__((address_space(3))) bf16x4* lds_frag_ptr;
template <int N>
__device__ __forceinline__ bf16x4 frag_at(lds_frag_ptr frag, int idx) {
  return frag[idx];
}

// Y[mt] = sum_kt F_dir[mt][kt] X[kt] (split-BF16 products, FP32 accumulation)
template <int N>
__device__ __forceinline__ void dft_mfma(lds_frag_ptr frag, int dir, int lane, const f32x4* X, f32x4* Y) {
  constexpr int NT = ZMfma<N>::NT;
  bf16x4 xh[NT], xl[NT];
#pragma unroll
  for (int kt = 0; kt < NT; ++kt) split_bf16(X[kt], xh[kt], xl[kt]);
  // the NT output tiles are independent accumulation chains: interleave them to hide MFMA latency
#pragma unroll
  for (int mt = 0; mt < NT; ++mt) Y[mt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kt = 0; kt < NT; ++kt) {
    // beyond 4 x 4 tiles, keep the fragments of this stage out of registers across stages and
    // group iterations (a compiler-only fence: no instruction, nothing is loaded by it)
    if constexpr (NT > 4) asm volatile("" ::: "memory");
#pragma unroll
    for (int mt = 0; mt < NT; ++mt)
      Y[mt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(frag_at<N>(frag, ZMfma<N>::frag(dir, 0, mt, kt) + lane),
                                                       xh[kt], Y[mt], 0, 0, 0);
#pragma unroll
    for (int mt = 0; mt < NT; ++mt)
      Y[mt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(frag_at<N>(frag, ZMfma<N>::frag(dir, 0, mt, kt) + lane),
                                                       xl[kt], Y[mt], 0, 0, 0);
#pragma unroll
    for (int mt = 0; mt < NT; ++mt)
      Y[mt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(frag_at<N>(frag, ZMfma<N>::frag(dir, 1, mt, kt) + lane),
                                                       xh[kt], Y[mt], 0, 0, 0);
  }
}

// complex helpers on the two values (z0, z0 + 1) a lane holds in one tile: (x, y) and (z, w)
__device__ __forceinline__ f32x4 cscale(const f32x4& v, float a, float b) {   // (a v0, b v1)
  return f32x4{a * v.x, a * v.y, b * v.z, b * v.w};
}
__device__ __forceinline__ f32x4 imul_scale(const f32x4& v, float a, float b) {   // (i a v0, i b v1)
  return f32x4{-a * v.y, a * v.x, -b * v.w, b * v.z};
}

// occupancy target at 24 points: 2 waves per SIMD for the many-to-one stages, 3 for the others
template <int N, int OP>
constexpr int kZMfmaWaves = N == 24 ? ((OP == OP_A2 || OP == OP_B) ? 2 : 3) : 1;

template <int N, int OP>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(kZMfmaWaves<N, OP>)))
k_zconv_mfma(const cx<float>* in, cx<float>* out, long npairs, int t0, MeshInfo mi, Tables tb,
             int sign_target_minus_partner, const bf16x4* frag_g, const cx<float>* inB = nullptr) {
  using Z = ZMfma<N>;
  constexpr int NT = Z::NT, NN = N * N, GPP = NN / 16;   // column groups per pair
  constexpr long NR = long(N) * N * N;
  constexpr int NIN = OpShape<OP>::nin, NOUT = OpShape<OP>::nout;
  __shared__ bf16x4 frag_sm[Z::NFRAG];
  for (int e = threadIdx.x; e < Z::NFRAG; e += blockDim.x) frag_sm[e] = frag_g[e];
  __syncthreads();
  const lds_frag_ptr frag = (lds_frag_ptr)(frag_sm);
  // register budget: the next group's inputs are prefetched only up to 4 x 4 tiles
  constexpr bool kPrefetch = NT <= 4;
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64, g4 = lane / 16, jc = lane % 16;
  const long ngroups = npairs * GPP;
  const long stride = long(gridDim.x) * 4;
  // lane's z values in tile m: z0 = 8 m + 2 g4 and z0 + 1
  auto load_col = [&](const cx<float>* b, f32x4* X) {
#pragma unroll
    for (int m = 0; m < NT; ++m) {
      const int z0 = 8 * m + 2 * g4;
      const cx<float> a = b[z0 * NN], c = b[(z0 + 1) * NN];
      X[m] = f32x4{a.x, a.y, c.x, c.y};
    }
  };
  auto store_col = [&](cx<float>* b, const f32x4* Yv) {
#pragma unroll
    for (int m = 0; m < NT; ++m) {
      const int z0 = 8 * m + 2 * g4;
      b[z0 * NN] = mk<float>(Yv[m].x, Yv[m].y);
      b[(z0 + 1) * NN] = mk<float>(Yv[m].z, Yv[m].w);
    }
  };
  auto col_base = [&](long grp, long& pair, int& xy) {
    pair = grp / GPP;
    xy = int(grp - pair * GPP) * 16 + jc;
  };
  // inputs of the next column group are loaded while this one is transformed
  f32x4 pre[NIN][NT];
  auto fetch = [&](long grp) {
    long pair;
    int xy;
    col_base(grp, pair, xy);
    if constexpr (NIN == 1) {
      int tt, qq;
      pair_tq(mi, t0, pair, tt, qq);
      load_col(in + (long(tt) * mi.P + qq) * NR + xy, pre[0]);
    } else {
#pragma unroll
      for (int c = 0; c < NIN; ++c) load_col(in + (pair * NIN + c) * NR + xy, pre[c]);
    }
    if constexpr (OP == OP_A2) {
      if (inB) {   // parallel inputs minus the pass-B sources
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          f32x4 b[NT];
          load_col(inB + (pair * 2 + c) * NR + xy, b);
#pragma unroll
          for (int m = 0; m < NT; ++m) pre[c][m] -= b[m];
        }
      }
    }
  };
  long grp = long(blockIdx.x) * 4 + wave;
  if (kPrefetch && grp < ngroups) fetch(grp);
  for (; grp < ngroups; grp += stride) {
    long pair;
    int xy;
    col_base(grp, pair, xy);
    if (!kPrefetch) fetch(grp);
    const bool more = kPrefetch && grp + stride < ngroups;
    int t, q;
    pair_tq(mi, t0, pair, t, q);
    const int di = pair_dindex(mi, t0 + t, q, sign_target_minus_partner);
    const float* tV = reinterpret_cast<const float*>(tb.V) + long(di) * NR + xy;
    const float* tU[2] = {reinterpret_cast<const float*>(tb.U1) + long(di) * NR + xy,
                          reinterpret_cast<const float*>(tb.U2) + long(di) * NR + xy};
    const float d3 = float(tb.dfr[3 * di + 2]);
    auto kap3 = [&](int z) { return float(mfreq<N>(z)) + d3; };
    f32x4 Y[NT], V[NT], O[NT];
    if constexpr (NIN == 1) {
      dft_mfma<N>(frag, 0, lane, pre[0], Y);
      if (more) fetch(grp + stride);   // the inputs are consumed: load the next group's
      cx<float>* ob = out + pair * NOUT * NR + xy;
      if constexpr (OP == OP_A1) {
#pragma unroll
        for (int m = 0; m < NT; ++m) {
          const int z0 = 8 * m + 2 * g4;
          V[m] = cscale(Y[m], tV[z0 * NN], tV[(z0 + 1) * NN]);
        }
        dft_mfma<N>(frag, 1, lane, V, O);
        store_col(ob, O);
        ob += NR;
      }
#pragma unroll 1
      for (int s = 0; s < 2; ++s) {
        float u0[NT], u1[NT];
#pragma unroll
        for (int m = 0; m < NT; ++m) {
          const int z0 = 8 * m + 2 * g4;
          u0[m] = tU[s][z0 * NN];
          u1[m] = tU[s][(z0 + 1) * NN];
          V[m] = cscale(Y[m], u0[m], u1[m]);
        }
        dft_mfma<N>(frag, 1, lane, V, O);
        store_col(ob, O);
#pragma unroll
        for (int m = 0; m < NT; ++m) {
          const int z0 = 8 * m + 2 * g4;
          V[m] = imul_scale(Y[m], kap3(z0) * u0[m], kap3(z0 + 1) * u1[m]);
        }
        dft_mfma<N>(frag, 1, lane, V, O);
        store_col(ob + NR, O);
        ob += 2 * NR;
      }
    } else {
#pragma unroll
      for (int m = 0; m < NT; ++m) V[m] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int s = 0; s < NIN / 2; ++s) {
        dft_mfma<N>(frag, 0, lane, pre[2 * s], Y);
#pragma unroll
        for (int m = 0; m < NT; ++m) {
          const int z0 = 8 * m + 2 * g4;
          V[m] += cscale(Y[m], tU[s][z0 * NN], tU[s][(z0 + 1) * NN]);
        }
        dft_mfma<N>(frag, 0, lane, pre[2 * s + 1], Y);
#pragma unroll
        for (int m = 0; m < NT; ++m) {
          const int z0 = 8 * m + 2 * g4;
          V[m] += cscale(Y[m], kap3(z0) * tU[s][z0 * NN], kap3(z0 + 1) * tU[s][(z0 + 1) * NN]);
        }
      }
      if (more) fetch(grp + stride);   // the inputs are consumed: load the next group's
      // OP_A2: -i acc; OP_B: +i acc
#pragma unroll
      for (int m = 0; m < NT; ++m) V[m] = OP == OP_A2 ? imul_scale(V[m], -1.f, -1.f) : imul_scale(V[m], 1.f, 1.f);
      dft_mfma<N>(frag, 1, lane, V, O);
      store_col(out + pair * NR + xy, O);
    }
  }
}

// Pass A, fused inverse xy + partner sums.  buf5 per pair (xy in G space):
// [XV, W0_par, W3_par, W0_anti, W3_anti]; after the inverse xy transform the lattice components Y_d
// of the vector fields are in LDS (Cartesian X_c = sum_d B_dc Y_d).  Accumulates for the owned points
// of target t over the chunk's partners q, with Dl = B D and Hl = B H3a4 (lattice components):
//   slot 0: -m2ax w XV psi_q                (2ax)
//   slot 1: -m2bx1 w X_par . D_q = -m2bx1 w Y_par . Dl_q      (2bx1)
//   slot 2: -m3a4 w H3a4_q . X_par = -m3a4 w Hl_q . Y_par     (2 x 3a4)
//   h4    : w X_par psi_q  (accumulated as w Y_par psi_q, made Cartesian at the end)   (Alg. 3a3)
// and, if do3b6, writes the 3b6 sources S_s,c = X_s,c n in the forward split form
// (lattice T_s = B S_s = M (n Y_s), M = B B^T) src4 per pair [P_par, R_par, P_anti, R_anti].  The metric
// is applied after the forward transform (it is constant): with U~_e the transform of n Y_s,e,
// P = sum_e (kappa_1 M_1e + kappa_2 M_2e) U~_e and R = sum_e M_3e U~_e.
// Delta = k_t - k_q.
template <typename R, int N>
struct PassA {
  static constexpr bool SPLIT = !Fz<R, N>::fits(7);   // spin channels in separate LDS rounds
  static constexpr int NPL = SPLIT ? 4 : 7;
};

// occupancy target: 3 waves per SIMD where that costs no spills (FP32 at 24^3)
template <typename R, int N>
constexpr int kFusedAWaves = (sizeof(R) == 4 && N == 24) ? 3 : 1;

// POL (spin-polarised runs): the antiparallel-channel 3b6 sources take the other spin's density nA.
// CN: the density is complex (biorthogonal mode, n = sum w conj(chi) psi); otherwise only its real part is
// read (n = sum w |psi|^2).
// H5A (TC mode, the orbitals as targets, pair store): h5[t] += w_q (|V_par|^2 + |V_anti|^2) (Alg. 3a2) into
// h5part ([S][T][N^3], real) in place of h4.  The occupied pass's V of the pair (a = t, b = q) is the conjugate
// of this pair's real-space fields (its density is the conjugate, its shift the negative), so the norms are
// the same, and its H3a4[t] = sum_q w_q conj(V_par) psi_q equals h4[t], which the caller takes from there.
// With POL the parallel and antiparallel parts of h5 are kept apart ([2][S][T][N^3]), as in k_fused_O.
template <typename R, int N, bool POL = false, bool CN = true, bool H5A = false>
__global__ void __launch_bounds__((Fz<R, N>::NTH)) __attribute__((amdgpu_waves_per_eu(kFusedAWaves<R, N>)))
k_fused_A(const cx<R>* buf5, const cx<R>* psi, const cx<R>* Dl, const cx<R>* Hl, const cx<R>* n, const double* w,
          FusedArgs fa, Masks m, int do3b6, MeshInfo mi, Basis<R> B, Basis<R> M, const double* dfr, cx<R>* src4,
          cx<R>* gpart, cx<R>* h4part, const cx<R>* nA = nullptr, const cx<R>* store = nullptr, int Q1 = 0,
          int tri = 0, int formed = 1, R* h5part = nullptr) {
  using F = Fz<R, N>;
  constexpr int KP = F::KP, RB = F::RB, PL = F::PLANE;
  constexpr bool SPLIT = PassA<R, N>::SPLIT;
  constexpr bool PF = !SPLIT && F::PREFETCH_A;
  constexpr long NR = long(N) * N * N;
  __shared__ cx<R> sm[PassA<R, N>::NPL * PL];
  const PlaneWG<R, N> wg(fa);
  const int jt = fa.t0 + wg.t;
  cx<R> ga[KP][3], h4[KP][3], nk[KP], na[POL ? KP : 1];
  R h5k[H5A ? KP : 1], h5ka[(H5A && POL) ? KP : 1];
  // |X|^2 of a Cartesian vector from its lattice components Y: Y^H M Y with the metric M = B B^T
  auto norm2 = [&](const cx<R>* Y) {
    R v = M.b[0] * (Y[0].x * Y[0].x + Y[0].y * Y[0].y) + M.b[4] * (Y[1].x * Y[1].x + Y[1].y * Y[1].y) +
          M.b[8] * (Y[2].x * Y[2].x + Y[2].y * Y[2].y);
    v += R(2) * (M.b[1] * (Y[0].x * Y[1].x + Y[0].y * Y[1].y) + M.b[2] * (Y[0].x * Y[2].x + Y[0].y * Y[2].y) +
                 M.b[5] * (Y[1].x * Y[2].x + Y[1].y * Y[2].y));
    return v;
  };
  unsigned ob[KP];   // byte offsets of the owned points within a volume
#pragma unroll
  for (int i = 0; i < KP; ++i) ob[i] = (wg.zo + RB * N * i) * unsigned(sizeof(cx<R>));
#pragma unroll
  for (int i = 0; i < KP; ++i) {
#pragma unroll
    for (int s = 0; s < 3; ++s) ga[i][s] = h4[i][s] = mk<R>(R(0), R(0));
    if constexpr (H5A) h5k[i] = R(0);
    if constexpr (H5A && POL) h5ka[i] = R(0);
    nk[i] = ldo(n, ob[i]);
    if constexpr (POL) na[i] = ldo(nA, ob[i]);
  }
  // 2bx1 is accumulated (into its own slot) whenever 2bx1 or 2bx2 is selected: its bracket is also the
  // energy of 2bx2, which pass B fuses with three-body terms
  const R a0 = R(-m.m2ax), a1 = R((m.m2bx1 != 0 || m.m2bx2 != 0) ? -1 : 0), a2 = R(-m.m3a4);
  // the next partner's five pair planes are loaded into registers while this partner is transformed
  cx<R> pre[5][KP];
  // the five pass-A planes of pair (jt, q): from the resident store, square ([target][Q1][5], partners
  // q < Q1) or triangular (tri: the pairs of q <= jt directly, those of q > jt through (q, jt), cj, while
  // jt < Q1); the others from the batch's own z stage ([t][P - Q1][5]; formed: it holds them for partners
  // q >= Q1)
  auto pairsrc = [&](int q, bool& cj) -> const cx<R>* {
    cj = false;
    if (tri) {
      if (q <= jt && q < Q1) return store + (tri_row(jt, Q1) + q) * 5 * NR;
      if (jt < Q1 && (q < Q1 || !formed)) {
        cj = true;
        return store + (tri_row(q, Q1) + jt) * 5 * NR;
      }
    } else if (q < Q1) {
      return store + (long(jt) * Q1 + q) * 5 * NR;
    }
    return buf5 + (long(wg.t) * (fa.P - Q1) + (q - Q1)) * 5 * NR;
  };
  // A reflected pair (cj) is loaded as the stored pair (q, jt) itself and transformed with that pair's
  // shift (the negative of (jt, q)'s): its real-space fields are the conjugates of (jt, q)'s, and are
  // conjugated where they are read after the inverse transforms.  The loads are the same for both cases.
  auto fetch = [&](int q) {
    bool cj;
    const gptr<cx<R>> src = uniform_global(pairsrc(q, cj));
#pragma unroll
    for (int f = 0; f < 5; ++f)
#pragma unroll
      for (int i = 0; i < KP; ++i) pre[f][i] = ldo(src + f * NR, ob[i]);
  };
  if (PF && wg.qb < wg.qe) fetch(wg.qb);
  for (int q = wg.qb; q < wg.qe; ++q) {
    const R wq = R(w[q]);
    const long pair = long(wg.t) * fa.P + q;
    const double* dl = dfr + 3 * pair_dindex(mi, jt, q, 1);
    const double del[2] = {ld_uniform(dl), ld_uniform(dl + 1)};
    const R k1 = R(double(mfreq<N>(wg.x)) + del[0]);
    bool cj;
    const cx<R>* src = pairsrc(q, cj);
    const double dsg = cj ? -1.0 : 1.0;   // shift of the loaded pair relative to (jt, q)
    const R k1l = R(double(mfreq<N>(wg.x)) + dsg * del[0]);
    // a value of the inverse-transformed planes, conjugated for a reflected pair
    auto rd = [&](int idx) {
      const cx<R> v = sm[idx];
      return mk<R>(v.x, cj ? -v.y : v.y);
    };
    const gptr<cx<R>> pq = uniform_global(psi + long(q) * NR);
    const gptr<cx<R>> dq = uniform_global(Dl + long(q) * NR);       // component d at dq + d P N^3
    const gptr<cx<R>> hq = uniform_global(Hl + long(q) * 3 * NR);   // component d at hq + d N^3
#pragma unroll 1
    for (int g = 0; g < (SPLIT ? 2 : 1); ++g) {
      const bool par = !SPLIT || g == 0, anti = !SPLIT || g == 1;
      const int ab = SPLIT ? 0 : 4;   // LDS slot of Y_anti,1
      // unsplit: the five planes are all requested before the first is used (left to itself the
      // compiler waits for each load in turn); split: each field is loaded where it is stored
      constexpr bool STAGE = !PF && !SPLIT;
      if constexpr (STAGE) fetch(q);
      auto field = [&](int f, int i) -> cx<R> {
        if constexpr (PF || STAGE)
          return pre[f][i];
        else
          return src[f * NR + wg.zo + RB * N * i];
      };
      // load: slot 0 XV, slots 1-3 Y_par, slots ab..ab+2 Y_anti
#pragma unroll
      for (int i = 0; i < KP; ++i) {
        const int so = wg.so0 + RB * F::LD * i;
        const R k2l = R(double(mfreq<N>(wg.y0 + RB * i)) + dsg * del[1]);
        if (par) {
          sm[so] = field(0, i);
          const cx<R> w0 = field(1, i);
          sm[PL + so] = mul_i(k1l * w0);
          sm[2 * PL + so] = mul_i(k2l * w0);
          sm[3 * PL + so] = field(2, i);
        }
        if (anti) {
          const cx<R> w0 = field(3, i);
          sm[ab * PL + so] = mul_i(k1l * w0);
          sm[(ab + 1) * PL + so] = mul_i(k2l * w0);
          sm[(ab + 2) * PL + so] = field(4, i);
        }
      }
      if (PF && q + 1 < wg.qe) fetch(q + 1);
      __syncthreads();
      planes_fft<R, N, 1>(sm, SPLIT ? (g == 0 ? 4 : 3) : 7, threadIdx.x);
#pragma unroll
      for (int i = 0; i < KP; ++i) {
        const unsigned r = wg.zo + RB * N * i;
        const int so = wg.ss(i);
        if (par) {
          const cx<R> p = ldo(pq, ob[i]);
          cfma(ga[i][0], a0 * wq, rd(so), p);
          cx<R> Y[3];
#pragma unroll
          for (int d = 0; d < 3; ++d) Y[d] = rd((1 + d) * PL + so);
          // the two dot products are summed over d before their weights are applied
          cx<R> sD = Y[0] * ldo(dq, ob[i]), sH = Y[0] * ldo(hq, ob[i]);
#pragma unroll
          for (int d = 1; d < 3; ++d) {
            sD = sD + Y[d] * ldo(dq + long(d) * fa.P * NR, ob[i]);
            sH = sH + Y[d] * ldo(hq + d * NR, ob[i]);
          }
          ga[i][1] = ga[i][1] + (a1 * wq) * sD;
          ga[i][2] = ga[i][2] + (a2 * wq) * sH;
          if constexpr (H5A) {
            h5k[i] += wq * norm2(Y);
          } else {
#pragma unroll
            for (int d = 0; d < 3; ++d) cfma(h4[i][d], wq, Y[d], p);
          }
          if (do3b6) {
#pragma unroll
            for (int d = 0; d < 3; ++d) sm[(1 + d) * PL + so] = CN ? Y[d] * nk[i] : nk[i].x * Y[d];
          }
        }
        if (anti && (do3b6 || H5A)) {
          cx<R> nanti;
          if constexpr (POL)
            nanti = na[i];
          else
            nanti = nk[i];
          cx<R> y[3];
#pragma unroll
          for (int d = 0; d < 3; ++d) y[d] = rd((ab + d) * PL + so);
          if constexpr (H5A && POL)
            h5ka[i] += wq * norm2(y);
          else if constexpr (H5A)
            h5k[i] += wq * norm2(y);
          if (do3b6) {
#pragma unroll
            for (int d = 0; d < 3; ++d) sm[(ab + d) * PL + so] = CN ? y[d] * nanti : nanti.x * y[d];
          }
        }
      }
      // finish this partner's multiply-accumulates here (a compiler-only fence: no instruction), so that
      // the partner fields loaded for them are not kept live across the forward transforms
#pragma unroll
      for (int i = 0; i < KP; ++i)
#pragma unroll
        for (int s = 0; s < 3; ++s) {
          if constexpr (H5A)
            asm volatile("" : "+v"(ga[i][s].x), "+v"(ga[i][s].y));
          else
            asm volatile("" : "+v"(ga[i][s].x), "+v"(ga[i][s].y), "+v"(h4[i][s].x), "+v"(h4[i][s].y));
        }
#pragma unroll
      for (int i = 0; i < (H5A ? KP : 0); ++i) asm volatile("" : "+v"(h5k[i]));
#pragma unroll
      for (int i = 0; i < ((H5A && POL) ? KP : 0); ++i) asm volatile("" : "+v"(h5ka[i]));
      __syncthreads();
      if (do3b6) {
        // forward xy of the T planes (slots 1..6 unsplit; 1..3 or 0..2 split), then the split form
        const int s0 = (SPLIT && g == 1) ? 0 : 1;
        planes_fft<R, N, -1, true>(sm + s0 * PL, SPLIT ? 3 : 6, threadIdx.x);
        cx<R>* dst = src4 + pair * 4 * NR;
#pragma unroll
        for (int i = 0; i < KP; ++i) {
          const int so = wg.so0 + RB * F::LD * i;
          const R k2 = R(double(mfreq<N>(wg.y0 + RB * i)) + del[1]);
          R c[3];   // kappa_1 M_1e + kappa_2 M_2e
#pragma unroll
          for (int e = 0; e < 3; ++e) c[e] = k1 * M.b[e] + k2 * M.b[3 + e];
          auto emit = [&](int slot, cx<R>* d0) {
            const cx<R> u0 = sm[slot * PL + so], u1 = sm[(slot + 1) * PL + so], u2 = sm[(slot + 2) * PL + so];
            sto(d0, ob[i], c[0] * u0 + c[1] * u1 + c[2] * u2);
            sto(d0 + NR, ob[i], M.b[6] * u0 + M.b[7] * u1 + M.b[8] * u2);
          };
          if (par) emit(1, dst);
          if (anti) emit(ab, dst + 2 * NR);
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < KP; ++i) {
    const unsigned r = wg.zo + RB * N * i;
    cx<R> hc[3];
    to_cart(B, h4[i], hc);
    cx<R>* gp = gpart + (long(wg.c) * fa.T + wg.t) * 3 * NR;
    cx<R>* hp = h4part + (long(wg.c) * fa.T + wg.t) * 3 * NR;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      sto(gp + s * NR, ob[i], ga[i][s]);
      if constexpr (!H5A) sto(hp + s * NR, ob[i], hc[s]);
    }
    if constexpr (H5A) sto(h5part + (long(wg.c) * fa.T + wg.t) * NR, ob[i] / unsigned(sizeof(cx<R>) / sizeof(R)), h5k[i]);
    if constexpr (H5A && POL)
      sto(h5part + (long(fa.S + wg.c) * fa.T + wg.t) * NR, ob[i] / unsigned(sizeof(cx<R>) / sizeof(R)), h5ka[i]);
  }
}

// One field per pair (xy in G space): partial of coef sum_q w_q Y psi_q, GRP partners per round.
template <typename R, int N>
__global__ void __launch_bounds__((Fz<R, N>::NTH)) __attribute__((amdgpu_waves_per_eu(Fz<R, N>::WAVES1)))
k_fused_Y(const cx<R>* buf1, const cx<R>* psi, const double* w,
                                                           FusedArgs fa, double coef, cx<R>* gpart) {
  using F = Fz<R, N>;
  constexpr int KP = F::KP, RB = F::RB;
  constexpr long NR = long(N) * N * N;
  __shared__ cx<R> sm[F::GRP1 * F::PLANE];
  const PlaneWG<R, N> wg(fa);
  cx<R> ga[KP];
#pragma unroll
  for (int i = 0; i < KP; ++i) ga[i] = mk<R>(R(0), R(0));
  for (int q0 = wg.qb; q0 < wg.qe; q0 += F::GRP1) {
    const int nq = min(F::GRP1, wg.qe - q0);
    for (int cc = 0; cc < nq; ++cc) {
      const cx<R>* src = buf1 + (long(wg.t) * fa.P + q0 + cc) * NR + wg.zo;
#pragma unroll
      for (int i = 0; i < KP; ++i) sm[cc * F::PLANE + wg.so0 + RB * F::LD * i] = src[RB * N * i];
    }
    __syncthreads();
    planes_fft<R, N, 1, true>(sm, nq, threadIdx.x);
#pragma unroll
    for (int i = 0; i < KP; ++i) {
      const long r = wg.zo + RB * N * i;
      const int so = wg.ss(i);
      for (int cc = 0; cc < nq; ++cc)
        cfma(ga[i], R(coef * w[q0 + cc]), sm[cc * F::PLANE + so], psi[long(q0 + cc) * NR + r]);
    }
    wg.end_round();
  }
#pragma unroll
  for (int i = 0; i < KP; ++i) gpart[(long(wg.c) * fa.T + wg.t) * NR + wg.zo + RB * N * i] = ga[i];
}

// Occupied-occupied pass: buf4 per pair (a = t0 + t, b = q; Delta = k_b - k_a), xy in G space:
// [W0_par, W3_par, W0_anti, W3_anti] at field offset (t sT + q sQ) N^3 (sT < 0: the pair-major layout
// sT = 4P, sQ = 4 of the pass's own z stage).  With V_s the Cartesian vector fields:
//   h5[a]   += w_b (|V_par|^2 + |V_anti|^2)     (Alg. 3a2; TC mode: V_ba = conj(V_ab))
//   H3a4[a] += w_b conj(V_par) psi_b            (Alg. 3a4 h3; Alg. 3b2 h3 is its conjugate)
template <typename R, int N>
struct PassO {
  static constexpr bool SPLIT = !Fz<R, N>::fits(6);
  static constexpr int NPL = SPLIT ? 3 : 6;
};

// SPLITH (spin-polarised runs): the parallel- and antiparallel-channel parts of h5 are kept apart, the
// antiparallel one in the second half of h5part ([2][S][T][N^3]); they serve targets of the partners' own
// spin and of the other spin respectively.
// H5 = false: only H3a4, from the parallel channel's three planes (h5part is written as zeros); in TC mode
// with the pair store, pass A accumulates h5 of every target from the same fields (k_fused_A<H5A>).
// In FP32 at 48 points the parallel-only form (three planes, 56 KB of LDS) runs two 768-thread work-groups per
// CU at 80 registers, without the register prefetch (measured faster than one work-group with it).
template <typename R, int N, bool H5>
constexpr int kFusedOWaves = (!H5 && Fz<R, N>::TWO_WG) ? 6 : 1;
template <typename R, int N, bool SPLITH = false, bool H5 = true>
__global__ void __launch_bounds__((Fz<R, N>::NTH)) __attribute__((amdgpu_waves_per_eu(kFusedOWaves<R, N, H5>)))
k_fused_O(const cx<R>* buf4, const cx<R>* psi, const double* w, FusedArgs fa, MeshInfo mi, Recip rc,
          const double* dfr, R* h5part, cx<R>* H3part, long sT = -1, long sQ = 4, const cx<R>* trs = nullptr,
          int Q1 = 0) {
  using F = Fz<R, N>;
  constexpr int KP = F::KP, RB = F::RB, PL = F::PLANE;
  constexpr bool SPLIT = H5 && PassO<R, N>::SPLIT;
  constexpr bool PF = !SPLIT && F::PREFETCH && (H5 || !F::TWO_WG);
  constexpr int NF = H5 ? 4 : 2;   // pair fields read: W0, W3 of the parallel channel (and the antiparallel)
  if (sT < 0) sT = 4L * fa.P;
  constexpr long NR = long(N) * N * N;
  __shared__ cx<R> sm[(H5 ? PassO<R, N>::NPL : 3) * PL];
  const PlaneWG<R, N> wg(fa);
  const Basis<R> B = basis<R>(rc);
  // |X|^2 of a Cartesian vector X_c = sum_d B_dc Y_d from its lattice components: Y^H M Y with the metric
  // M = B B^T (diagonal Md, twice the off-diagonal Mo for the pairs 12, 13, 23)
  R Md[3], Mo[3];
#pragma unroll
  for (int d = 0; d < 3; ++d)
    Md[d] = B.b[3 * d] * B.b[3 * d] + B.b[3 * d + 1] * B.b[3 * d + 1] + B.b[3 * d + 2] * B.b[3 * d + 2];
  Mo[0] = R(2) * (B.b[0] * B.b[3] + B.b[1] * B.b[4] + B.b[2] * B.b[5]);
  Mo[1] = R(2) * (B.b[0] * B.b[6] + B.b[1] * B.b[7] + B.b[2] * B.b[8]);
  Mo[2] = R(2) * (B.b[3] * B.b[6] + B.b[4] * B.b[7] + B.b[5] * B.b[8]);
  auto norm2 = [&](const cx<R>* Y) {
    return Md[0] * (Y[0].x * Y[0].x + Y[0].y * Y[0].y) + Md[1] * (Y[1].x * Y[1].x + Y[1].y * Y[1].y) +
           Md[2] * (Y[2].x * Y[2].x + Y[2].y * Y[2].y) + Mo[0] * (Y[0].x * Y[1].x + Y[0].y * Y[1].y) +
           Mo[1] * (Y[0].x * Y[2].x + Y[0].y * Y[2].y) + Mo[2] * (Y[1].x * Y[2].x + Y[1].y * Y[2].y);
  };
  const int ja = fa.t0 + wg.t;
  R h5[KP], h5b[SPLITH ? KP : 1];
  cx<R> H[KP][3];   // lattice components (conj(X_c) = sum_d B_dc conj(Y_d)), made Cartesian at the end
#pragma unroll
  for (int i = 0; i < KP; ++i) {
    h5[i] = R(0);
    if constexpr (SPLITH) h5b[i] = R(0);
    H[i][0] = H[i][1] = H[i][2] = mk<R>(R(0), R(0));
  }
  // fields 1..4 of the pair (row ja, partner q): at t sT + q sQ in buf4, or (trs, the triangular store of
  // pass-A pairs) the stored pair (q, ja) of ja <= q, else (cj) the stored pair (ja, q), which is loaded as it
  // is, transformed with its own shift (the negative) and conjugated in real space where it is read
  auto pairsrc = [&](int q, bool& cj) -> const cx<R>* {
    cj = false;
    if (trs) {
      if (ja <= q) return trs + ((tri_row(q, Q1) + ja) * 5 + 1) * NR;
      cj = true;
      return trs + ((tri_row(ja, Q1) + q) * 5 + 1) * NR;
    }
    return buf4 + (long(wg.t) * sT + long(q) * sQ) * NR;
  };
  auto ld = [&](const cx<R>* src, int f, int i) -> cx<R> {
    return ldo(uniform_global(src) + f * NR, (wg.zo + RB * N * i) * unsigned(sizeof(cx<R>)));
  };
  // the next partner's four pair planes are loaded into registers while this partner is transformed
  cx<R> pre[NF][KP];
  auto fetch = [&](int q) {
    bool cj;
    const gptr<cx<R>> src = uniform_global(pairsrc(q, cj));
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
      for (int i = 0; i < KP; ++i) pre[f][i] = ldo(src + f * NR, (wg.zo + RB * N * i) * unsigned(sizeof(cx<R>)));
  };
  if (PF && wg.qb < wg.qe) fetch(wg.qb);
  for (int q = wg.qb; q < wg.qe; ++q) {
    const R wq = R(w[q]);
    const double* dl = dfr + 3 * pair_dindex(mi, ja, q, 0);
    const double del[2] = {ld_uniform(dl), ld_uniform(dl + 1)};
    bool cj;
    const cx<R>* src = pairsrc(q, cj);
    const double dsg = cj ? -1.0 : 1.0;   // shift of the loaded pair relative to (q, ja)
    // grid frequencies (exact in R) recomputed per partner rather than held across the loop (compiler-only
    // fences); the shift rounded once to R
    int xx = wg.x, yy = wg.y0;
    asm volatile("" : "+v"(xx), "+v"(yy));
    const R k1 = R(mfreq<N>(xx)) + R(dsg * del[0]);
#pragma unroll 1
    for (int g = 0; g < (SPLIT ? 2 : 1); ++g) {
      const bool par = !SPLIT || g == 0, anti = H5 && (!SPLIT || g == 1);
      const int ab = SPLIT ? 0 : 3;
#pragma unroll
      for (int i = 0; i < KP; ++i) {
        const int so = wg.so0 + RB * F::LD * i;
        const R k2 = R(mfreq<N>(yy + RB * i)) + R(dsg * del[1]);
        if (par) {
          const cx<R> w0 = !PF ? ld(src, 0, i) : pre[0][i];
          sm[so] = mul_i(k1 * w0);
          sm[PL + so] = mul_i(k2 * w0);
          sm[2 * PL + so] = !PF ? ld(src, 1, i) : pre[1][i];
        }
        if constexpr (H5) {
          if (anti) {
            const cx<R> w0 = !PF ? ld(src, 2, i) : pre[2][i];
            sm[ab * PL + so] = mul_i(k1 * w0);
            sm[(ab + 1) * PL + so] = mul_i(k2 * w0);
            sm[(ab + 2) * PL + so] = !PF ? ld(src, 3, i) : pre[3][i];
          }
        }
      }
      if (PF && q + 1 < wg.qe) fetch(q + 1);
      __syncthreads();
      planes_fft<R, N, 1, true, kFusedOWaves<R, N, H5> != 1>(sm, (SPLIT || !H5) ? 3 : 6, threadIdx.x);
#pragma unroll
      for (int i = 0; i < KP; ++i) {
        const long r = wg.zo + RB * N * i;
        const int so = wg.ss(i);
        cx<R> Y[3];
        if (par) {
          const cx<R> pq = ldo(uniform_global(psi + long(q) * NR), unsigned(r) * unsigned(sizeof(cx<R>)));
#pragma unroll
          for (int d = 0; d < 3; ++d) Y[d] = sm[d * PL + so];
          if constexpr (H5) h5[i] += wq * norm2(Y);
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            const cx<R> hv = cmulc(mk<R>(Y[d].x, cj ? -Y[d].y : Y[d].y), pq);   // Y conjugated when reflected
            H[i][d].x += wq * hv.x;
            H[i][d].y += wq * hv.y;
          }
        }
        if (anti) {
#pragma unroll
          for (int d = 0; d < 3; ++d) Y[d] = sm[(ab + d) * PL + so];
          const R v = wq * norm2(Y);
          if constexpr (SPLITH)
            h5b[i] += v;
          else
            h5[i] += v;
        }
      }
      wg.end_round();
    }
  }
#pragma unroll
  for (int i = 0; i < KP; ++i) {
    const long r = wg.zo + RB * N * i;
    h5part[(long(wg.c) * fa.T + wg.t) * NR + r] = h5[i];
    if constexpr (SPLITH) h5part[(long(fa.S + wg.c) * fa.T + wg.t) * NR + r] = h5b[i];
    cx<R> Hc[3];
    to_cart(B, H[i], Hc);
#pragma unroll
    for (int cd = 0; cd < 3; ++cd) H3part[((long(wg.c) * fa.T + wg.t) * 3 + cd) * NR + r] = Hc[cd];
  }
}

// Occupied-occupied pass with left orbitals (biorthogonal mode), a = t0 + t (q2 of Algs. 3a2, 3a4, 3b2),
// b = q (q1).  V21 comes from rho21 = conj(chi_a) psi_b (Delta = k_b - k_a, buf21) and V12 from
// rho12 = conj(chi_b) psi_a (Delta = k_a - k_b, buf12); each holds [W0_par, W3_par, W0_anti, W3_anti] per
// pair, xy in G space.  With V the Cartesian vector fields:
//   h5[a]  += w_b sum_s V21_s . V12_s        (Alg. 3a2, bilinear; complex)
//   H3a4[a] += w_b V12_par psi_b              (Alg. 3a4 h3)
//   H3bc[a] += w_b conj(V21_par) chi_b        (conjugate of the h3 of Algs. 3b2 / 3b5)
template <typename R, int N>
struct PassOB {
  static constexpr bool SPLIT = !Fz<R, N>::fits(6);   // V21 and V12 in separate LDS rounds
  static constexpr int NPL = SPLIT ? 3 : 6;
  // register prefetch of the next round where it costs no spills (FP32 up to 16 points); at 24 points
  // the kernel runs at 3 waves per SIMD without it instead
  static constexpr bool PF = sizeof(R) == 4 && N <= 16;
  static constexpr int WAVES = (sizeof(R) == 4 && N == 24) ? 3 : 1;
};

// Field offsets (in N^3 units) of pair (row t of the batch, partner q): t sT + q sQ for V21 and for V12;
// sT < 0: the pair-major layout of the pass's own z stages (sT = 4P, sQ = 4).  With the resident store of
// pass-A z-stage outputs ([pair][5], fields 1..4 as here): V21 of (a, b) is stored pair (t = b, q = a) and
// V12 is stored pair (t = a, q = b).
// SPLITH (spin-polarised runs): the parallel- and antiparallel-channel parts of h5 are kept apart, the
// antiparallel one in the second half of h5part ([2][S][T][N^3]), as in k_fused_O.
template <typename R, int N, bool SPLITH = false>
__global__ void __launch_bounds__((Fz<R, N>::NTH)) __attribute__((amdgpu_waves_per_eu(PassOB<R, N>::WAVES)))
k_fused_OB(const cx<R>* buf21, const cx<R>* buf12,
                                                            const cx<R>* psi, const cx<R>* chi, const double* w,
                                                            FusedArgs fa, MeshInfo mi, Recip rc, const double* dfr,
                                                            cx<R>* h5part, cx<R>* H3part, cx<R>* Hbpart,
                                                            long sT21 = -1, long sQ21 = 4, long sT12 = -1,
                                                            long sQ12 = 4) {
  using F = Fz<R, N>;
  if (sT21 < 0) sT21 = 4L * fa.P;
  if (sT12 < 0) sT12 = 4L * fa.P;
  constexpr int KP = F::KP, RB = F::RB, PL = F::PLANE;
  constexpr bool SPLIT = PassOB<R, N>::SPLIT, PF = PassOB<R, N>::PF;
  constexpr long NR = long(N) * N * N;
  __shared__ cx<R> sm[PassOB<R, N>::NPL * PL];
  const PlaneWG<R, N> wg(fa);
  const Basis<R> B = basis<R>(rc);
  const int ja = fa.t0 + wg.t;
  cx<R> h5[KP], h5b[SPLITH ? KP : 1], H[KP][3], Hb[KP][3], X21[KP][3];
#pragma unroll
  for (int i = 0; i < KP; ++i) {
    h5[i] = mk<R>(R(0), R(0));
    if constexpr (SPLITH) h5b[i] = mk<R>(R(0), R(0));
#pragma unroll
    for (int c = 0; c < 3; ++c) H[i][c] = Hb[i][c] = mk<R>(R(0), R(0));
  }
  // One round per (partner q, spin channel ch): [W0, W3] of V21 and of V12 for that channel.  With PF the
  // next round's four planes (and, for a parallel-channel round, psi_q and chi_q at the owned points) are
  // loaded into registers while this round is transformed; otherwise at the start of each round.
  cx<R> pre[4][KP], pp[2][KP];
  auto fetch = [&](int q, int ch) {
    const cx<R>* s21 = buf21 + (long(wg.t) * sT21 + long(q) * sQ21) * NR + wg.zo;
    const cx<R>* s12 = buf12 + (long(wg.t) * sT12 + long(q) * sQ12) * NR + wg.zo;
#pragma unroll
    for (int i = 0; i < KP; ++i) {
      const long o = RB * N * i;
      pre[0][i] = s21[(2 * ch) * NR + o];
      pre[1][i] = s21[(2 * ch + 1) * NR + o];
      pre[2][i] = s12[(2 * ch) * NR + o];
      pre[3][i] = s12[(2 * ch + 1) * NR + o];
    }
    if (ch == 0) {
#pragma unroll
      for (int i = 0; i < KP; ++i) {
        pp[0][i] = psi[long(q) * NR + wg.zo + RB * N * i];
        pp[1][i] = chi[long(q) * NR + wg.zo + RB * N * i];
      }
    }
  };
  if (PF && wg.qb < wg.qe) fetch(wg.qb, 0);
  for (int q = wg.qb; q < wg.qe; ++q) {
    const R wq = R(w[q]);
    const double* del[2] = {dfr + 3 * pair_dindex(mi, ja, q, 0), dfr + 3 * pair_dindex(mi, ja, q, 1)};
#pragma unroll 1
    for (int ch = 0; ch < 2; ++ch) {   // spin channel of the kernel: parallel, antiparallel
      if (!PF) fetch(q, ch);
#pragma unroll 1
      for (int h = 0; h < (SPLIT ? 2 : 1); ++h) {
        // LDS: unsplit, slots 0-2 V21 and 3-5 V12; split, sub-round h holds field h in slots 0-2
#pragma unroll
        for (int v = 0; v < 2; ++v) {
          if (SPLIT && v != h) continue;
          const int base = SPLIT ? 0 : 3 * v;
          const R k1 = R(double(mfreq<N>(wg.x)) + del[v][0]);
#pragma unroll
          for (int i = 0; i < KP; ++i) {
            const int so = wg.so0 + RB * F::LD * i;
            const R k2 = R(double(mfreq<N>(wg.y0 + RB * i)) + del[v][1]);
            const cx<R> w0 = pre[2 * v][i];
            sm[base * PL + so] = mul_i(k1 * w0);
            sm[(base + 1) * PL + so] = mul_i(k2 * w0);
            sm[(base + 2) * PL + so] = pre[2 * v + 1][i];
          }
        }
        if (PF && (!SPLIT || h == 1)) {   // this round's planes are in LDS: load the next round's
          if (ch == 0)
            fetch(q, 1);
          else if (q + 1 < wg.qe)
            fetch(q + 1, 0);
        }
        __syncthreads();
        planes_fft<R, N, 1>(sm, SPLIT ? 3 : 6, threadIdx.x);
#pragma unroll
        for (int i = 0; i < KP; ++i) {
          const int so = wg.ss(i);
          cx<R> Y[3], X12[3];
          if (!SPLIT || h == 0) {
#pragma unroll
            for (int d = 0; d < 3; ++d) Y[d] = sm[d * PL + so];
            to_cart(B, Y, X21[i]);
          }
          if (!SPLIT || h == 1) {
            const int base = SPLIT ? 0 : 3;
#pragma unroll
            for (int d = 0; d < 3; ++d) Y[d] = sm[(base + d) * PL + so];
            to_cart(B, Y, X12);
            cx<R> hv = X21[i][0] * X12[0];
#pragma unroll
            for (int c = 1; c < 3; ++c) hv = hv + X21[i][c] * X12[c];
            if (SPLITH && ch == 1)
              h5b[i] = h5b[i] + wq * hv;
            else
              h5[i] = h5[i] + wq * hv;
            if (ch == 0) {
#pragma unroll
              for (int c = 0; c < 3; ++c) {
                H[i][c] = H[i][c] + wq * (X12[c] * pp[0][i]);
                Hb[i][c] = Hb[i][c] + wq * cmulc(X21[i][c], pp[1][i]);
              }
            }
          }
        }
        __syncthreads();
      }
    }
  }
#pragma unroll
  for (int i = 0; i < KP; ++i) {
    const long r = wg.zo + RB * N * i;
    const long o = long(wg.c) * fa.T + wg.t;
    h5part[o * NR + r] = h5[i];
    if constexpr (SPLITH) h5part[(long(fa.S + wg.c) * fa.T + wg.t) * NR + r] = h5b[i];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      H3part[(o * 3 + c) * NR + r] = H[i][c];
      Hbpart[(o * 3 + c) * NR + r] = Hb[i][c];
    }
  }
}

// Fixed-order FP64 sum of real partner-chunk partials: out[t0 + t] = sum_c parts[c][t]
template <typename R, int N>
__global__ void k_sum_real_parts(int S, int T, int t0, const R* parts, R* out) {
  constexpr long NR = long(N) * N * N;
  const long id = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id >= long(T) * NR) return;
  const int t = int(id / NR);
  const long r = id - long(t) * NR;
  double s = 0;
  for (int c = 0; c < S; ++c) s += double(parts[(long(c) * T + t) * NR + r]);
  out[long(t0 + t) * NR + r] = R(s);
}

// Fixed-order FP64 sum of complex partner-chunk partials: out[t0 + t] = sum_c parts[c][t]
template <typename R, int N>
__global__ void k_sum_cx_parts(int S, int T, int t0, const cx<R>* parts, cx<R>* out) {
  constexpr long NR = long(N) * N * N;
  const long id = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id >= long(T) * NR) return;
  const int t = int(id / NR);
  const long r = id - long(t) * NR;
  double sr = 0, si = 0;
  for (int c = 0; c < S; ++c) {
    const cx<R> v = parts[(long(c) * T + t) * NR + r];
    sr += double(v.x);
    si += double(v.y);
  }
  out[long(t0 + t) * NR + r] = mk<R>(R(sr), R(si));
}

// Fixed-order FP64 sums of the partials of k_fused_OB: h5[t0+t], H3a4[t0+t], H3bc[t0+t].
template <typename R, int N>
__global__ void k_sum_parts_ob(int S, int T, int t0, const cx<R>* h5part, const cx<R>* H3part,
                               const cx<R>* Hbpart, cx<R>* h5, cx<R>* H3a4, cx<R>* H3bc) {
  constexpr long NR = long(N) * N * N;
  const long id = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id >= long(T) * NR) return;
  const int t = int(id / NR);
  const long r = id - long(t) * NR;
  cx<double> s = {0, 0}, H[3] = {{0, 0}, {0, 0}, {0, 0}}, Hb[3] = {{0, 0}, {0, 0}, {0, 0}};
  for (int c = 0; c < S; ++c) {
    const long o = long(c) * T + t;
    const cx<R> v = h5part[o * NR + r];
    s.x += double(v.x);
    s.y += double(v.y);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const cx<R> a = H3part[(o * 3 + d) * NR + r], b = Hbpart[(o * 3 + d) * NR + r];
      H[d].x += double(a.x);
      H[d].y += double(a.y);
      Hb[d].x += double(b.x);
      Hb[d].y += double(b.y);
    }
  }
  h5[long(t0 + t) * NR + r] = mk<R>(R(s.x), R(s.y));
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    H3a4[(long(t0 + t) * 3 + d) * NR + r] = mk<R>(R(H[d].x), R(H[d].y));
    H3bc[(long(t0 + t) * 3 + d) * NR + r] = mk<R>(R(Hb[d].x), R(Hb[d].y));
  }
}

// Sum of the partner-chunk partials in a fixed order (FP64).
//   mode 0 (occ): h5[t0+t] = sum_c h5part, H3a4[t0+t] = sum_c H3part                  (working precision)
//   mode 1 (A)  : acc[s][t] += sum_c gpart[c][t][s] (s = 0,1,2), h4[t] = sum_c h4part
//   mode 2 (Y)  : acc[slot][t] += sum_c gpart[c][t]
template <typename R, int N>
__global__ void k_sum_parts(int mode, int S, int T, int t0, int slot, const R* h5part, const cx<R>* H3part,
                            const cx<R>* gpart, const cx<R>* h4part, R* h5, cx<R>* H3a4, cx<double>* acc, cx<R>* h4) {
  constexpr long NR = long(N) * N * N;
  const long id = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id >= long(T) * NR) return;
  const int t = int(id / NR);
  const long r = id - long(t) * NR;
  if (mode == 0) {
    double s = 0;
    cx<double> H[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (int c = 0; c < S; ++c) {
      s += double(h5part[(long(c) * T + t) * NR + r]);
#pragma unroll
      for (int cd = 0; cd < 3; ++cd) {
        const cx<R> v = H3part[((long(c) * T + t) * 3 + cd) * NR + r];
        H[cd].x += double(v.x);
        H[cd].y += double(v.y);
      }
    }
    h5[long(t0 + t) * NR + r] = R(s);
#pragma unroll
    for (int cd = 0; cd < 3; ++cd) H3a4[(long(t0 + t) * 3 + cd) * NR + r] = mk<R>(R(H[cd].x), R(H[cd].y));
  } else if (mode == 1) {
    cx<double> g[3] = {{0, 0}, {0, 0}, {0, 0}}, h[3] = {{0, 0}, {0, 0}, {0, 0}};
    for (int c = 0; c < S; ++c) {
#pragma unroll
      for (int s = 0; s < 3; ++s) {
        const cx<R> v = gpart[((long(c) * T + t) * 3 + s) * NR + r];
        g[s].x += double(v.x);
        g[s].y += double(v.y);
        if (h4part) {
          const cx<R> u = h4part[((long(c) * T + t) * 3 + s) * NR + r];
          h[s].x += double(u.x);
          h[s].y += double(u.y);
        }
      }
    }
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      cx<double>& a = acc[(long(s) * T + t) * NR + r];
      a.x += g[s].x;
      a.y += g[s].y;
      if (h4part) h4[(long(t) * 3 + s) * NR + r] = mk<R>(R(h[s].x), R(h[s].y));
    }
  } else {
    cx<double> g = {0, 0};
    for (int c = 0; c < S; ++c) {
      const cx<R> v = gpart[(long(c) * T + t) * NR + r];
      g.x += double(v.x);
      g.y += double(v.y);
    }
    cx<double>& a = acc[(long(slot) * T + t) * NR + r];
    a.x += g.x;
    a.y += g.y;
  }
}

// Local (Hartree-type) terms added to the FP64 accumulators, then g_t = sum of the slots that belong to
// the operator.  loc: [VH, h1 x3, P2bh2, F3b1, h6, F3b2]; D is stored component-major D[(c*P + p)*N^3 + r].
// acc slots (kAccSlots): 0 = 2ah + 2ax, 1 = 2bx1 (unit weight; enters g times the 2bx1 multiplier), 2 = three-body
// terms outside pass B, 3 = pass B (2bx2, 3b3, 3b4, 3b5, and 3b6 when selected with any of them), 4 = 2bh1,
// 5 = 2bh2.
constexpr int kAccSlots = 6;

template <typename R, int N>
__global__ void k_local(const cx<R>* psi, const cx<R>* D, const cx<R>* loc, const cx<R>* h4, int t0, int T, int P,
                        Masks m, cx<double>* acc, cx<R>* g) {
  constexpr long NR = long(N) * N * N;
  const long id = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id >= long(T) * NR) return;
  const int t = int(id / NR);
  const long r = id - long(t) * NR;
  const long j = t0 + t;
  const long TS = long(T) * NR;
  const cx<R> pj = psi[j * NR + r];
  const cx<R> VH = loc[r];
  cx<R> h1[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) h1[c] = loc[(1 + c) * NR + r];
  const cx<R> P2 = loc[4 * NR + r], F3b1 = loc[5 * NR + r], h6 = loc[6 * NR + r], F3b2 = loc[7 * NR + r];
  cx<R> hD = mk<R>(R(0), R(0)), hh = mk<R>(R(0), R(0)), h14 = mk<R>(R(0), R(0));
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    hD = hD + h1[c] * D[(long(c) * P + j) * NR + r];
    hh = hh + h1[c] * h1[c];
    h14 = h14 + h1[c] * h4[(long(t) * 3 + c) * NR + r];
  }
  const cx<R> s3 = R(-0.5 * m.m3a1) * hh - R(m.m3b1) * F3b1 + R(0.5 * m.m3a2) * h6 + R(m.m3b2) * F3b2;
  const cx<R> v[kAccSlots] = {(R(m.m2ah) * VH) * pj, mk<R>(R(0), R(0)), s3 * pj + R(m.m3a3) * h14,
                              mk<R>(R(0), R(0)), R(m.m2bh1) * hD, (R(m.m2bh2) * P2) * pj};
  double gx = 0, gy = 0;
#pragma unroll
  for (int s = 0; s < kAccSlots; ++s) {
    cx<double>& a = acc[s * TS + long(t) * NR + r];
    a.x += double(v[s].x);
    a.y += double(v[s].y);
    const double ws = s == 1 ? m.m2bx1 : 1.0;   // slot 1 holds 2bx1 with unit weight
    gx += ws * a.x;
    gy += ws * a.y;
  }
  g[long(t) * NR + r] = mk<R>(R(gx), R(gy));
}

// Energy partials: e[j*kAccSlots + slot] = Re sum_r conj(chi_j) acc_slot,t / N^3 (deterministic work-group
// sum, one block per (t, slot); chi = psi in TC mode)
template <typename R, int N>
__global__ void __launch_bounds__(256) k_epart(const cx<R>* chi, const cx<double>* acc, int t0, int T, double* e) {
  constexpr long NR = long(N) * N * N;
  const int t = blockIdx.x / kAccSlots, slot = blockIdx.x % kAccSlots;
  const cx<R>* p = chi + long(t0 + t) * NR;
  const cx<double>* a = acc + (long(slot) * T + t) * NR;
  double s = 0;
  for (long r = threadIdx.x; r < NR; r += blockDim.x) s += double(p[r].x) * a[r].x + double(p[r].y) * a[r].y;
  s = wg_sum(s);
  if (threadIdx.x == 0) e[long(t0 + t) * kAccSlots + slot] = s / double(NR);
}

// h6 = sum_a w_a h5[a];  M_c = sum_a w_a conj(H3c[a]_c) psi_a, H3c = conj(H3b) (Alg. 3b2 source;
// TC mode: H3c = H3a4 and h5 real)
__device__ __forceinline__ double re_part(float v) { return v; }
__device__ __forceinline__ double re_part(double v) { return v; }
__device__ __forceinline__ double im_part(float) { return 0.0; }
__device__ __forceinline__ double im_part(double) { return 0.0; }
template <typename R>
__device__ __forceinline__ double re_part(cx<R> v) { return double(v.x); }
template <typename R>
__device__ __forceinline__ double im_part(cx<R> v) { return double(v.y); }

template <typename R, int N, typename H5>
__global__ void k_reduce_occ(const H5* h5, const cx<R>* H3c, const cx<R>* psi, const double* w, int P, cx<R>* h6,
                             cx<R>* M) {
  constexpr long NR = long(N) * N * N;
  const long r = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= NR) return;
  double s = 0, si = 0, mr[3] = {0, 0, 0}, mi[3] = {0, 0, 0};
  for (int a = 0; a < P; ++a) {
    const H5 hv = h5[long(a) * NR + r];
    s += w[a] * re_part(hv);
    si += w[a] * im_part(hv);
    const cx<R> pa = psi[long(a) * NR + r];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const cx<R> v = cmulc(H3c[(long(a) * 3 + c) * NR + r], pa);
      mr[c] += w[a] * double(v.x);
      mi[c] += w[a] * double(v.y);
    }
  }
  h6[r] = mk<R>(R(s), R(si));
#pragma unroll
  for (int c = 0; c < 3; ++c) M[c * NR + r] = mk<R>(R(mr[c]), R(mi[c]));
}

// 3a2 with h5 from pass A (k_fused_A<H5A>), applied after every target batch: h6 = sum_a w_a h5_a (fixed-order
// FP64 sum, as in k_reduce_occ) ...
template <typename R, int N>
__global__ void k_h6_sum(const R* h5, const double* w, int P, cx<R>* h6) {
  constexpr long NR = long(N) * N * N;
  const long r = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= NR) return;
  double s = 0;
  for (int a = 0; a < P; ++a) s += w[a] * double(h5[long(a) * NR + r]);
  h6[r] = mk<R>(R(s), R(0));
}
// ... then per target batch g_t = coef h6 psi_j (coef = m3a2 / 2, the local 3a2 term that k_local leaves out
// on this path), for the r -> G transform and a gather that adds it to the output ...
template <typename R, int N>
__global__ void k_h6_apply(const cx<R>* psi, const cx<R>* h6, int t0, int T, R coef, cx<R>* g) {
  constexpr long NR = long(N) * N * N;
  const long id = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id >= long(T) * NR) return;
  const int t = int(id / NR);
  const long r = id - long(t) * NR;
  g[long(t) * NR + r] = (coef * h6[r]) * psi[long(t0 + t) * NR + r];
}
// ... and its energy, added to the three-body slot: e[j kAccSlots + slot] += Re sum_r conj(psi_j) coef h6 psi_j / N^3
// (one work-group per target, deterministic sum)
template <typename R, int N>
__global__ void __launch_bounds__(256) k_h6_energy(const cx<R>* psi, const cx<R>* h6, int t0, double coef, int slot,
                                                   double* e) {
  constexpr long NR = long(N) * N * N;
  const int j = t0 + int(blockIdx.x);
  const cx<R>* p = psi + long(j) * NR;
  double s = 0;
  for (long r = threadIdx.x; r < NR; r += blockDim.x) {
    const double a = double(p[r].x), b = double(p[r].y);
    s += double(h6[r].x) * (a * a + b * b);
  }
  s = wg_sum(s);
  if (threadIdx.x == 0) e[long(j) * kAccSlots + slot] += coef * s / double(NR);
}

// Pass-B target factor in lattice components: Zl_t = B (m2bx2 D_j - m3b3 h1 psi_j + m3b4 h4_t)
template <typename R, int N>
__global__ void k_passB_Z(const cx<R>* psi, const cx<R>* D, const cx<R>* h1, const cx<R>* h4, int t0, int T, int P,
                          Masks m, Basis<R> B, cx<R>* Zl) {
  constexpr long NR = long(N) * N * N;
  const long id = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id >= long(T) * NR) return;
  const int t = int(id / NR);
  const long r = id - long(t) * NR;
  const long j = t0 + t;
  const cx<R> pj = psi[j * NR + r];
  cx<R> Zc[3], Zd[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    cx<R> v = R(m.m2bx2) * D[(long(c) * P + j) * NR + r];
    v = v - R(m.m3b3) * (h1[c * NR + r] * pj);
    v = v + R(m.m3b4) * h4[(long(t) * 3 + c) * NR + r];
    Zc[c] = v;
  }
  to_latt(B, Zc, Zd);
#pragma unroll
  for (int d = 0; d < 3; ++d) Zl[(long(t) * 3 + d) * NR + r] = Zd[d];
}

}  // namespace tcmi
