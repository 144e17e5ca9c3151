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

namespace tcmi {

struct Recip {
  double b[9];   // rows b1, b2, b3 (cartesian, bohr^-1)
};

struct MeshInfo {
  int n1, n2, n3;   // k-mesh
  int nb;           // bands per k-point
  int P;            // orbitals of one spin channel (nk * nb)
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
                         double scale, double* out, long nr) {
  const long t = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= long(nt) * npw_max) return;
  const int jt = int(t / npw_max), g = int(t - long(jt) * npw_max);
  const int j = j0 + jt;
  const int ik = j / nb;
  double re = 0, im = 0;
  if (g < npw[ik]) {
    const cx<R> v = f[long(jt) * nr + boxidx[long(ik) * npw_max + g]];
    re = double(v.x) * scale;
    im = double(v.y) * scale;
  }
  out[2 * (long(j) * npw_max + g)] = re;
  out[2 * (long(j) * npw_max + g) + 1] = im;
}

// ---------------------------------------------------------------- densities (TC: chi = phi)
// n = sum_q w_q |psi_q|^2, J_c = sum_q w_q conj(psi_q) D_qc, accumulated in FP64.
template <typename R, int N>
__global__ void k_density(const cx<R>* psi, const cx<R>* D, const double* w, int P, cx<R>* n, cx<R>* J) {
  constexpr long NR = long(N) * N * N;
  const long r = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= NR) return;
  double nn = 0, jr[3] = {0, 0, 0}, ji[3] = {0, 0, 0};
  for (int q = 0; q < P; ++q) {
    const cx<R> a = psi[q * NR + r];
    const double wq = w[q];
    nn += wq * (double(a.x) * a.x + double(a.y) * a.y);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const cx<R> d = D[(long(c) * P + q) * NR + r];
      jr[c] += wq * (double(a.x) * d.x + double(a.y) * d.y);
      ji[c] += wq * (double(a.x) * d.y - double(a.y) * d.x);
    }
  }
  n[r] = mk<R>(R(nn), R(0));
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

// ---------------------------------------------------------------- pair passes
// Forward xy transform of pair densities rho = conj(X[ix]) Y[iy].
// TFIRST: ix = t0 + t, iy = q (occupied-occupied pass, rho_ab = conj(chi_a) psi_b);
// else   ix = q, iy = t0 + t  (target passes, rho_qj = conj(chi_q) psi_j).
template <typename R, int N, bool TFIRST>
struct IOPair {
  const cx<R>* X;
  const cx<R>* Y;
  cx<R>* out;
  int t0, P;
  __device__ cx<R> load(long pl, int y, int x) const {
    constexpr long NR = long(N) * N * N;
    const long pair = pl / N;
    const int z = int(pl - pair * N);
    const int t = int(pair / P), q = int(pair - long(t) * P);
    const long ix = TFIRST ? t0 + t : q, iy = TFIRST ? q : t0 + t;
    const long o = long(z) * N * N + y * N + x;
    return cmulc(X[ix * NR + o], Y[iy * NR + o]);
  }
  __device__ void store(long pl, int y, int x, cx<R> v) const { out[pl * N * N + y * N + x] = v; }
};

template <typename R, int N, bool TFIRST>
__global__ void __launch_bounds__(256) k_xy_pair(const cx<R>* X, const cx<R>* Y, cx<R>* out, int t0, int P,
                                                 long nplanes) {
  IOPair<R, N, TFIRST> io{X, Y, out, t0, P};
  xy_block<R, N, -1>(io, nplanes);
}

// Pass-B sources: Y_c = conj(psi_q) Z_tc + m3b5 * H3b_qc * psi_j, H3b = conj(H3a4) (TC mode);
// Z holds D_j - h1 psi_j + h4_j (masked) per target.
template <typename R, int N>
struct IOPassB {
  const cx<R>* psi;
  const cx<R>* Z;
  const cx<R>* H3a4;
  cx<R>* out;
  int t0, P;
  R m3b5;
  __device__ cx<R> load(long pl, int y, int x) const {
    constexpr long NR = long(N) * N * N;
    const long f = pl / N;              // pair*3 + c
    const int z = int(pl - f * N);
    const long pair = f / 3;
    const int c = int(f - pair * 3);
    const int t = int(pair / P), q = int(pair - long(t) * P);
    const long o = long(z) * N * N + y * N + x;
    const cx<R> pq = psi[long(q) * NR + o];
    cx<R> v = cmulc(pq, Z[(long(t) * 3 + c) * NR + o]);
    if (m3b5 != R(0)) v = v + m3b5 * cmulc(H3a4[(long(q) * 3 + c) * NR + o], psi[long(t0 + t) * NR + o]);
    return v;
  }
  __device__ void store(long pl, int y, int x, cx<R> v) const { out[pl * N * N + y * N + x] = v; }
};

template <typename R, int N>
__global__ void __launch_bounds__(256) k_xy_passB(const cx<R>* psi, const cx<R>* Z, const cx<R>* H3a4, cx<R>* out,
                                                  int t0, int P, R m3b5, long nplanes) {
  IOPassB<R, N> io{psi, Z, H3a4, out, t0, P, m3b5};
  xy_block<R, N, -1>(io, nplanes);
}

// z stage of a pair convolution: forward z transform of the inputs, kernel multiply
// at Q = Delta + G for the pair's Delta, inverse z transform of each output.
//   OP_A1: 1 -> 7   [V2a_par rho, iQ u_par rho (3), iQ u_anti rho (3)]
//   OP_O : 1 -> 6   [iQ u_par rho (3), iQ u_anti rho (3)]
//   OP_A2: 6 -> 1   sum_c -iQ_c (u_par S_par,c + u_anti S_anti,c)
//   OP_B : 3 -> 1   sum_c  iQ_c u_par Y_c
enum { OP_A1 = 0, OP_O = 1, OP_A2 = 2, OP_B = 3 };

template <int OP>
struct OpShape;
template <> struct OpShape<OP_A1> { static constexpr int nin = 1, nout = 7; };
template <> struct OpShape<OP_O> { static constexpr int nin = 1, nout = 6; };
template <> struct OpShape<OP_A2> { static constexpr int nin = 6, nout = 1; };
template <> struct OpShape<OP_B> { static constexpr int nin = 3, nout = 1; };

struct Tables {
  const void* V;    // V2a (parallel), exchange conventions, [nDelta][N^3]
  const void* U1;   // u~ parallel
  const void* U2;   // u~ antiparallel
  const double* dfr;  // [nDelta][3] fractions of Delta
};

template <typename R, int N, int OP>
__global__ void __launch_bounds__(256) k_zconv(const cx<R>* in, cx<R>* out, long npairs, int t0, MeshInfo mi,
                                               Recip rc, Tables tb, int sign_target_minus_partner) {
  constexpr int NN = N * N;
  constexpr long NR = long(N) * N * N;
  constexpr int NIN = OpShape<OP>::nin, NOUT = OpShape<OP>::nout;
  const long col = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (col >= npairs * NN) return;
  const long pair = col / NN;
  const int xy = int(col - pair * NN);
  const int x = xy % N, y = xy / N;
  const int t = int(pair / mi.P), q = int(pair - long(t) * mi.P);
  const int kt = (t0 + t) / mi.nb, kq = q / mi.nb;
  const int di = sign_target_minus_partner ? kindex_delta(mi, kt, kq) : kindex_delta(mi, kq, kt);
  const R* tV = reinterpret_cast<const R*>(tb.V) + long(di) * NR;
  const R* tU1 = reinterpret_cast<const R*>(tb.U1) + long(di) * NR;
  const R* tU2 = reinterpret_cast<const R*>(tb.U2) + long(di) * NR;
  const double* dfr = tb.dfr + 3 * di;

  cx<R> acc[N];
  if constexpr (NIN == 1) {
    const cx<R>* b = in + pair * NR + xy;
#pragma unroll
    for (int z = 0; z < N; ++z) acc[z] = b[z * NN];
    fft_line<R, N, -1>(acc);
  } else {
#pragma unroll
    for (int z = 0; z < N; ++z) acc[z] = mk<R>(R(0), R(0));
#pragma unroll 1
    for (int c = 0; c < NIN; ++c) {
      cx<R> v[N];
      const cx<R>* b = in + (pair * NIN + c) * NR + xy;
#pragma unroll
      for (int z = 0; z < N; ++z) v[z] = b[z * NN];
      fft_line<R, N, -1>(v);
#pragma unroll
      for (int z = 0; z < N; ++z) {
        R Q[3];
        qvec<R, N>(rc, dfr, x, y, z, Q);
        const long o = long(z) * NN + xy;
        if constexpr (OP == OP_A2) {
          const int s = c / 3, cc = c - 3 * (c / 3);
          const R u = s == 0 ? tU1[o] : tU2[o];
          acc[z] = acc[z] + mul_i((-Q[cc] * u) * v[z]);
        } else {  // OP_B
          acc[z] = acc[z] + mul_i((Q[c] * tU1[o]) * v[z]);
        }
      }
    }
  }
  if constexpr (NOUT == 1) {
    fft_line<R, N, 1>(acc);
    cx<R>* b = out + pair * NR + xy;
#pragma unroll
    for (int z = 0; z < N; ++z) b[z * NN] = acc[z];
  } else {
#pragma unroll 1
    for (int o = 0; o < NOUT; ++o) {
      cx<R> v[N];
#pragma unroll
      for (int z = 0; z < N; ++z) {
        const long oo = long(z) * NN + xy;
        if constexpr (OP == OP_A1) {
          if (o == 0) {
            v[z] = tV[oo] * acc[z];
          } else {
            R Q[3];
            qvec<R, N>(rc, dfr, x, y, z, Q);
            const int s = (o - 1) / 3, cc = (o - 1) - 3 * ((o - 1) / 3);
            const R u = s == 0 ? tU1[oo] : tU2[oo];
            v[z] = mul_i((Q[cc] * u) * acc[z]);
          }
        } else {  // OP_O
          R Q[3];
          qvec<R, N>(rc, dfr, x, y, z, Q);
          const int s = o / 3, cc = o - 3 * (o / 3);
          const R u = s == 0 ? tU1[oo] : tU2[oo];
          v[z] = mul_i((Q[cc] * u) * acc[z]);
        }
      }
      fft_line<R, N, 1>(v);
      cx<R>* b = out + (pair * NOUT + o) * NR + xy;
#pragma unroll
      for (int z = 0; z < N; ++z) b[z * NN] = v[z];
    }
  }
}

// ---------------------------------------------------------------- masks
struct Masks {
  double m2ah, m2bh1, m2bh2, m2ax, m2bx1, m2bx2, m3a1, m3a2, m3a3, m3a4, m3b1, m3b2, m3b3, m3b4, m3b5, m3b6;
};

// ---------------------------------------------------------------- fused inverse-xy + partner sums
// A work-group owns one target t, one z-plane and one chunk of partners.  For
// every partner it loads the z-stage outputs of the pair (xy still in G space),
// finishes the 3D inverse transform with an in-LDS xy transform and accumulates
// the pair's contributions for the N^2 points of its plane in registers.
// Thread layout: RB rows x N columns; thread (y0, x) owns the points (y0 + RB i, x)
// and, in the transform passes, one line.  Partner sums run in the working
// precision inside a chunk (<= 64 partners) and in FP64 across chunks.
template <typename R, int N>
struct Fz {
  static constexpr int RB = (N % 8 == 0) ? 8 : 4;
  static constexpr int NTH = RB * N;                                    // threads per work-group
  static constexpr int KP = N / RB;                                     // owned points per thread
  static constexpr int LD = N + 1;
  static constexpr int PLANE = N * LD;                                  // LDS elements per plane
  static constexpr int kBudget = 65536;
  static constexpr int kFit = kBudget / int(PLANE * sizeof(cx<R>));
  static constexpr int GRP0 = kFit < 1 ? 1 : kFit;
  static constexpr int GRP = GRP0 < RB ? GRP0 : RB;                    // planes in LDS at once (<= RB lines/thread)
};

// in-place 2D transform of np <= RB planes in LDS ([np][N][N+1]); ends with a barrier
template <typename R, int N, int DIR>
__device__ __forceinline__ void planes_fft(cx<R>* sm, int np, int tid) {
  constexpr int LD = N + 1;
  const int p = tid / N, l = tid - (tid / N) * N;
  const bool act = p < np;
  if (act) {
    cx<R> v[N];
    cx<R>* row = sm + (p * N + l) * LD;
#pragma unroll
    for (int x = 0; x < N; ++x) v[x] = row[x];
    fft_line<R, N, DIR>(v);
#pragma unroll
    for (int x = 0; x < N; ++x) row[x] = v[x];
  }
  __syncthreads();
  if (act) {
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

struct FusedArgs {
  int P, T, t0, S, chunk;     // orbitals, targets in batch, first target, partner chunks, partners per chunk
};

template <typename R>
__device__ __forceinline__ void cfma(cx<R>& acc, R a, cx<R> u, cx<R> v) {   // acc += a u v
  const cx<R> p = u * v;
  acc.x += a * p.x;
  acc.y += a * p.y;
}

// Pass A: buf7 per pair [XV, XU_par(3), XU_anti(3)] (xy in G space).  Slots:
//   0: -m2ax w XV psi_q          (2ax)
//   1: -m2bx1 w XU . D_q         (2bx1)
//   2: -m3a4 w H3a4_q . XU       (2 x 3a4)
//   h4 += w XU psi_q             (h4 of Alg. 3a3)
// and, if do3b6, writes the 3b6 sources S_{s,c} = X^{U,s}_c n, forward xy transformed.
template <typename R, int N>
__global__ void __launch_bounds__((Fz<R, N>::NTH)) k_fused_A(const cx<R>* buf7, const cx<R>* psi, const cx<R>* D,
                                                           const cx<R>* H3a4, const cx<R>* n, const double* w,
                                                           FusedArgs fa, Masks m, int do3b6, cx<R>* src6,
                                                           cx<R>* gpart, cx<R>* h4part) {
  using F = Fz<R, N>;
  constexpr int NN = N * N, KP = F::KP, RB = F::RB;
  constexpr long NR = long(N) * N * N;
  __shared__ cx<R> sm[F::GRP * F::PLANE];
  const int tid = threadIdx.x;
  const int x = tid % N, y0 = tid / N;
  const int c = blockIdx.x % fa.S;
  const int z = (blockIdx.x / fa.S) % N;
  const int t = blockIdx.x / (fa.S * N);
  const int qb = c * fa.chunk, qe = min(fa.P, qb + fa.chunk);
  const long zo = long(z) * NN + y0 * N + x;      // global offset of owned point i: zo + RB*N*i
  const int so0 = y0 * F::LD + x;                 // LDS offset of owned point i: so0 + RB*LD*i
  cx<R> ga[KP][3], h4[KP][3], nk[KP];
#pragma unroll
  for (int i = 0; i < KP; ++i) {
#pragma unroll
    for (int s = 0; s < 3; ++s) ga[i][s] = h4[i][s] = mk<R>(R(0), R(0));
    nk[i] = n[zo + RB * N * i];
  }
  const R a0 = R(-m.m2ax), a1 = R(-m.m2bx1), a2 = R(-m.m3a4);
  for (int q = qb; q < qe; ++q) {
    const R wq = R(w[q]);
    const long pair = long(t) * fa.P + q;
    for (int c0 = 0; c0 < 7; c0 += F::GRP) {
      const int nc = min(F::GRP, 7 - c0);
      for (int cc = 0; cc < nc; ++cc) {
        const cx<R>* src = buf7 + (pair * 7 + c0 + cc) * NR + zo;
#pragma unroll
        for (int i = 0; i < KP; ++i) sm[cc * F::PLANE + so0 + RB * F::LD * i] = src[RB * N * i];
      }
      __syncthreads();
      planes_fft<R, N, 1>(sm, nc, tid);
#pragma unroll
      for (int i = 0; i < KP; ++i) {
        const long r = zo + RB * N * i;
        const int so = so0 + RB * F::LD * i;
        const cx<R> pq = psi[long(q) * NR + r];
#pragma unroll
        for (int comp = 0; comp < 7; ++comp) {
          if (comp < c0 || comp >= c0 + nc) continue;
          cx<R>* slot = sm + (comp - c0) * F::PLANE + so;
          const cx<R> X = *slot;
          if (comp == 0) {
            cfma(ga[i][0], a0 * wq, X, pq);
          } else if (comp <= 3) {
            const int cd = comp - 1;
            cfma(ga[i][1], a1 * wq, X, D[(long(cd) * fa.P + q) * NR + r]);
            cfma(ga[i][2], a2 * wq, X, H3a4[(long(q) * 3 + cd) * NR + r]);
            cfma(h4[i][cd], wq, X, pq);
            *slot = X * nk[i];
          } else {
            *slot = X * nk[i];
          }
        }
      }
      __syncthreads();
      if (do3b6) {
        const int s0 = c0 == 0 ? 1 : 0;     // component 0 (XV) has no 3b6 source
        planes_fft<R, N, -1>(sm + s0 * F::PLANE, nc - s0, tid);
        for (int cc = s0; cc < nc; ++cc) {
          cx<R>* dst = src6 + (pair * 6 + c0 + cc - 1) * NR + zo;
#pragma unroll
          for (int i = 0; i < KP; ++i) dst[RB * N * i] = sm[cc * F::PLANE + so0 + RB * F::LD * i];
        }
        __syncthreads();
      }
    }
  }
#pragma unroll
  for (int i = 0; i < KP; ++i) {
    const long r = zo + RB * N * i;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      gpart[((long(c) * fa.T + t) * 3 + s) * NR + r] = ga[i][s];
      h4part[((long(c) * fa.T + t) * 3 + s) * NR + r] = h4[i][s];
    }
  }
}

// One field per pair (xy in G space): partial of coef sum_q w_q Y psi_q.  GRP partners at a time.
template <typename R, int N>
__global__ void __launch_bounds__((Fz<R, N>::NTH)) k_fused_Y(const cx<R>* buf1, const cx<R>* psi, const double* w,
                                                           FusedArgs fa, double coef, cx<R>* gpart) {
  using F = Fz<R, N>;
  constexpr int NN = N * N, KP = F::KP, RB = F::RB;
  constexpr long NR = long(N) * N * N;
  __shared__ cx<R> sm[F::GRP * F::PLANE];
  const int tid = threadIdx.x;
  const int x = tid % N, y0 = tid / N;
  const int c = blockIdx.x % fa.S;
  const int z = (blockIdx.x / fa.S) % N;
  const int t = blockIdx.x / (fa.S * N);
  const int qb = c * fa.chunk, qe = min(fa.P, qb + fa.chunk);
  const long zo = long(z) * NN + y0 * N + x;
  const int so0 = y0 * F::LD + x;
  cx<R> ga[KP];
#pragma unroll
  for (int i = 0; i < KP; ++i) ga[i] = mk<R>(R(0), R(0));
  for (int q0 = qb; q0 < qe; q0 += F::GRP) {
    const int nq = min(F::GRP, qe - q0);
    for (int cc = 0; cc < nq; ++cc) {
      const cx<R>* src = buf1 + (long(t) * fa.P + q0 + cc) * NR + zo;
#pragma unroll
      for (int i = 0; i < KP; ++i) sm[cc * F::PLANE + so0 + RB * F::LD * i] = src[RB * N * i];
    }
    __syncthreads();
    planes_fft<R, N, 1>(sm, nq, tid);
#pragma unroll
    for (int i = 0; i < KP; ++i) {
      const long r = zo + RB * N * i;
      const int so = so0 + RB * F::LD * i;
#pragma unroll
      for (int cc = 0; cc < F::GRP; ++cc) {
        if (cc >= nq) continue;
        cfma(ga[i], R(coef * w[q0 + cc]), sm[cc * F::PLANE + so], psi[long(q0 + cc) * NR + r]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < KP; ++i) gpart[(long(c) * fa.T + t) * NR + zo + RB * N * i] = ga[i];
}

// Occupied-occupied pass: buf6 per pair (a = t0+t, b = q) [V_par(3), V_anti(3)], xy in G space.
//   h5[a]   += w_b (|V_par|^2 + |V_anti|^2)     (Alg. 3a2; TC mode: V_ba = conj(V_ab))
//   H3a4[a] += w_b conj(V_par) psi_b            (Alg. 3a4 h3; Alg. 3b2 h3 is its conjugate)
template <typename R, int N>
__global__ void __launch_bounds__((Fz<R, N>::NTH)) k_fused_O(const cx<R>* buf6, const cx<R>* psi, const double* w,
                                                           FusedArgs fa, R* h5part, cx<R>* H3part) {
  using F = Fz<R, N>;
  constexpr int NN = N * N, KP = F::KP, RB = F::RB;
  constexpr long NR = long(N) * N * N;
  __shared__ cx<R> sm[F::GRP * F::PLANE];
  const int tid = threadIdx.x;
  const int x = tid % N, y0 = tid / N;
  const int c = blockIdx.x % fa.S;
  const int z = (blockIdx.x / fa.S) % N;
  const int t = blockIdx.x / (fa.S * N);
  const int qb = c * fa.chunk, qe = min(fa.P, qb + fa.chunk);
  const long zo = long(z) * NN + y0 * N + x;
  const int so0 = y0 * F::LD + x;
  R h5[KP];
  cx<R> H[KP][3];
#pragma unroll
  for (int i = 0; i < KP; ++i) {
    h5[i] = R(0);
    H[i][0] = H[i][1] = H[i][2] = mk<R>(R(0), R(0));
  }
  for (int q = qb; q < qe; ++q) {
    const R wq = R(w[q]);
    const long pair = long(t) * fa.P + q;
    for (int c0 = 0; c0 < 6; c0 += F::GRP) {
      const int nc = min(F::GRP, 6 - c0);
      for (int cc = 0; cc < nc; ++cc) {
        const cx<R>* src = buf6 + (pair * 6 + c0 + cc) * NR + zo;
#pragma unroll
        for (int i = 0; i < KP; ++i) sm[cc * F::PLANE + so0 + RB * F::LD * i] = src[RB * N * i];
      }
      __syncthreads();
      planes_fft<R, N, 1>(sm, nc, tid);
#pragma unroll
      for (int i = 0; i < KP; ++i) {
        const long r = zo + RB * N * i;
        const int so = so0 + RB * F::LD * i;
        const cx<R> pq = psi[long(q) * NR + r];
#pragma unroll
        for (int comp = 0; comp < 6; ++comp) {
          if (comp < c0 || comp >= c0 + nc) continue;
          const cx<R> V = sm[(comp - c0) * F::PLANE + so];
          h5[i] += wq * (V.x * V.x + V.y * V.y);
          if (comp < 3) {
            const cx<R> hv = cmulc(V, pq);
            H[i][comp].x += wq * hv.x;
            H[i][comp].y += wq * hv.y;
          }
        }
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int i = 0; i < KP; ++i) {
    const long r = zo + RB * N * i;
    h5part[(long(c) * fa.T + t) * NR + r] = h5[i];
#pragma unroll
    for (int cd = 0; cd < 3; ++cd) H3part[((long(c) * fa.T + t) * 3 + cd) * NR + r] = H[i][cd];
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
        const cx<R> u = h4part[((long(c) * T + t) * 3 + s) * NR + r];
        g[s].x += double(v.x);
        g[s].y += double(v.y);
        h[s].x += double(u.x);
        h[s].y += double(u.y);
      }
    }
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      cx<double>& a = acc[(long(s) * T + t) * NR + r];
      a.x += g[s].x;
      a.y += g[s].y;
      h4[(long(t) * 3 + s) * NR + r] = mk<R>(R(h[s].x), R(h[s].y));
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

// Local (Hartree-type) terms added to the FP64 accumulators, then g_t = sum of the four slots.
// loc: [VH, h1 x3, P2bh2, F3b1, h6, F3b2]; D is stored component-major D[(c*P + p)*N^3 + r].
// acc slots: 0 = 2ah/2ax, 1 = 2bh1/2bx1, 2 = other three-body terms, 3 = pass B + 2bh2.
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
  const cx<R> v[4] = {(R(m.m2ah) * VH) * pj, R(m.m2bh1) * hD, s3 * pj + R(m.m3a3) * h14, (R(m.m2bh2) * P2) * pj};
  double gx = 0, gy = 0;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    cx<double>& a = acc[s * TS + long(t) * NR + r];
    a.x += double(v[s].x);
    a.y += double(v[s].y);
    gx += a.x;
    gy += a.y;
  }
  g[long(t) * NR + r] = mk<R>(R(gx), R(gy));
}

// Energy partials: e[j*4 + slot] = Re sum_r conj(psi_j) acc_slot,t / N^3 (deterministic tree, one block per (t, slot))
template <typename R, int N>
__global__ void __launch_bounds__(256) k_epart(const cx<R>* psi, const cx<double>* acc, int t0, int T, double* e) {
  constexpr long NR = long(N) * N * N;
  const int t = blockIdx.x / 4, slot = blockIdx.x % 4;
  const cx<R>* p = psi + long(t0 + t) * NR;
  const cx<double>* a = acc + (long(slot) * T + t) * NR;
  double s = 0;
  for (long r = threadIdx.x; r < NR; r += blockDim.x) s += double(p[r].x) * a[r].x + double(p[r].y) * a[r].y;
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (int(threadIdx.x) < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) e[long(t0 + t) * 4 + slot] = red[0] / double(NR);
}

// h6 = sum_a w_a h5[a];  M_c = sum_a w_a conj(H3a4[a]_c) psi_a  (H3b = conj(H3a4) in TC mode)
template <typename R, int N>
__global__ void k_reduce_occ(const R* h5, const cx<R>* H3a4, const cx<R>* psi, const double* w, int P, cx<R>* h6,
                             cx<R>* M) {
  constexpr long NR = long(N) * N * N;
  const long r = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= NR) return;
  double s = 0, mr[3] = {0, 0, 0}, mi[3] = {0, 0, 0};
  for (int a = 0; a < P; ++a) {
    s += w[a] * double(h5[long(a) * NR + r]);
    const cx<R> pa = psi[long(a) * NR + r];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const cx<R> v = cmulc(H3a4[(long(a) * 3 + c) * NR + r], pa);
      mr[c] += w[a] * double(v.x);
      mi[c] += w[a] * double(v.y);
    }
  }
  h6[r] = mk<R>(R(s), R(0));
#pragma unroll
  for (int c = 0; c < 3; ++c) M[c * NR + r] = mk<R>(R(mr[c]), R(mi[c]));
}

// Z_t = m2bx2 D_j - m3b3 h1 psi_j + m3b4 h4_t  (pass-B target factor)
template <typename R, int N>
__global__ void k_passB_Z(const cx<R>* psi, const cx<R>* D, const cx<R>* h1, const cx<R>* h4, int t0, int T, int P,
                          Masks m, cx<R>* Z) {
  constexpr long NR = long(N) * N * N;
  const long id = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id >= long(T) * NR) return;
  const int t = int(id / NR);
  const long r = id - long(t) * NR;
  const long j = t0 + t;
  const cx<R> pj = psi[j * NR + r];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    cx<R> v = R(m.m2bx2) * D[(long(c) * P + j) * NR + r];
    v = v - R(m.m3b3) * (h1[c * NR + r] * pj);
    v = v + R(m.m3b4) * h4[(long(t) * 3 + c) * NR + r];
    Z[(long(t) * 3 + c) * NR + r] = v;
  }
}

}  // namespace tcmi
