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

// Sources of the 3b6 chain: S_{s,c} = X^{U,s}_c * n for s in {par, anti}; buf7 holds
// [XV, XU_par x3, XU_anti x3] in real space per pair; output [pair][6][N^3], forward xy.
template <typename R, int N>
struct IO3b6 {
  const cx<R>* buf7;
  const cx<R>* n;
  cx<R>* out;
  __device__ cx<R> load(long pl, int y, int x) const {
    constexpr long NR = long(N) * N * N;
    const long f = pl / N;              // pair*6 + comp
    const int z = int(pl - f * N);
    const long pair = f / 6;
    const int comp = int(f - pair * 6);
    const long o = long(z) * N * N + y * N + x;
    return buf7[(pair * 7 + 1 + comp) * NR + o] * n[o];
  }
  __device__ void store(long pl, int y, int x, cx<R> v) const { out[pl * N * N + y * N + x] = v; }
};

template <typename R, int N>
__global__ void __launch_bounds__(256) k_xy_3b6(const cx<R>* buf7, const cx<R>* n, cx<R>* out, long nplanes) {
  IO3b6<R, N> io{buf7, n, out};
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

// ---------------------------------------------------------------- partner sums (FP64)
struct Masks {
  double m2ah, m2bh1, m2bh2, m2ax, m2bx1, m2bx2, m3a1, m3a2, m3a3, m3a4, m3b1, m3b2, m3b3, m3b4, m3b5, m3b6;
};

// Pass A, first stage.  buf7 (real space) per pair: [XV, XU_par(3), XU_anti(3)].
// acc layout [4][T][N^3] complex128: 0 = 2ah/2ax, 1 = 2bh1/2bx1, 2 = three-body, 3 = pass B/2bh2.
template <typename R, int N>
__global__ void k_acc_A1(const cx<R>* buf7, const cx<R>* psi, const cx<R>* D, const cx<R>* H3a4, const double* w,
                         int P, int T, Masks mk_, cx<double>* acc, cx<R>* h4) {
  constexpr long NR = long(N) * N * N;
  const long id = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id >= long(T) * NR) return;
  const int t = int(id / NR);
  const long r = id - long(t) * NR;
  double a0r = 0, a0i = 0, a1r = 0, a1i = 0, a2r = 0, a2i = 0;
  double hr[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  for (int q = 0; q < P; ++q) {
    const cx<R>* b = buf7 + (long(t) * P + q) * 7 * NR + r;
    const double wq = w[q];
    const cx<R> pq = psi[long(q) * NR + r];
    const cx<R> XV = b[0];
    const cx<R> v = XV * pq;
    a0r -= wq * double(v.x);
    a0i -= wq * double(v.y);
    cx<R> sd = mk<R>(R(0), R(0)), sh = mk<R>(R(0), R(0));
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const cx<R> XU = b[(1 + c) * NR];
      sd = sd + XU * D[(long(c) * P + q) * NR + r];
      sh = sh + XU * H3a4[(long(q) * 3 + c) * NR + r];
      const cx<R> hv = XU * pq;
      hr[c] += wq * double(hv.x);
      hi[c] += wq * double(hv.y);
    }
    a1r -= wq * double(sd.x);
    a1i -= wq * double(sd.y);
    a2r -= wq * double(sh.x);
    a2i -= wq * double(sh.y);
  }
  cx<double>* A0 = acc + long(t) * NR + r;
  const long TS = long(T) * NR;
  A0[0].x += mk_.m2ax * a0r;
  A0[0].y += mk_.m2ax * a0i;
  A0[TS].x += mk_.m2bx1 * a1r;
  A0[TS].y += mk_.m2bx1 * a1i;
  A0[2 * TS].x += mk_.m3a4 * a2r;
  A0[2 * TS].y += mk_.m3a4 * a2i;
#pragma unroll
  for (int c = 0; c < 3; ++c) h4[(long(t) * 3 + c) * NR + r] = mk<R>(R(hr[c]), R(hi[c]));
}

// acc[slot][t] += sign * sum_q w_q Y_tq psi_q   (Y: one field per pair, real space)
template <typename R, int N>
__global__ void k_acc_Y(const cx<R>* Y, const cx<R>* psi, const double* w, int P, int T, double coef, int slot,
                        cx<double>* acc) {
  constexpr long NR = long(N) * N * N;
  const long id = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id >= long(T) * NR) return;
  const int t = int(id / NR);
  const long r = id - long(t) * NR;
  double ar = 0, ai = 0;
  for (int q = 0; q < P; ++q) {
    const cx<R> v = Y[(long(t) * P + q) * NR + r] * psi[long(q) * NR + r];
    ar += w[q] * double(v.x);
    ai += w[q] * double(v.y);
  }
  cx<double>* A = acc + long(slot) * T * NR + long(t) * NR + r;
  A->x += coef * ar;
  A->y += coef * ai;
}

// Occupied-occupied pass: buf6 per pair (a = t0+t, b = q): [V_par(3), V_anti(3)], real space.
// h5[a] = sum_b w_b (|V_par|^2 + |V_anti|^2)   (TC mode: V_ba = conj(V_ab), Alg. 3a2)
// H3a4[a]_c = sum_b w_b conj(V_par,c) psi_b    (Alg. 3a4 h3; Alg. 3b2 h3 = conj of it)
template <typename R, int N>
__global__ void k_acc_O(const cx<R>* buf6, const cx<R>* psi, const double* w, int P, int T, int t0, R* h5,
                        cx<R>* H3a4) {
  constexpr long NR = long(N) * N * N;
  const long id = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id >= long(T) * NR) return;
  const int t = int(id / NR);
  const long r = id - long(t) * NR;
  double s5 = 0, hr[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  for (int q = 0; q < P; ++q) {
    const cx<R>* b = buf6 + (long(t) * P + q) * 6 * NR + r;
    const double wq = w[q];
    const cx<R> pq = psi[long(q) * NR + r];
    double s = 0;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const cx<R> v = b[c * NR];
      s += double(v.x) * v.x + double(v.y) * v.y;
      if (c < 3) {
        const cx<R> hv = cmulc(v, pq);
        hr[c] += wq * double(hv.x);
        hi[c] += wq * double(hv.y);
      }
    }
    s5 += wq * s;
  }
  h5[long(t0 + t) * NR + r] = R(s5);
#pragma unroll
  for (int c = 0; c < 3; ++c) H3a4[(long(t0 + t) * 3 + c) * NR + r] = mk<R>(R(hr[c]), R(hi[c]));
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

// Local (Hartree-type) terms, then g_t = sum of the four accumulators (working precision).
// D is stored component-major: D[(c*P + p)*N^3 + r].
// loc: [VH, h1 x3, P2bh2, F3b1, h6, F3b2] real-space fields
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
  const cx<R> t0v = (R(m.m2ah) * VH) * pj;
  const cx<R> t1v = R(m.m2bh1) * hD;
  const cx<R> t3v = (R(m.m2bh2) * P2) * pj;
  const cx<R> t2v = s3 * pj + R(m.m3a3) * h14;
  cx<double>* A = acc + long(t) * NR + r;
  A[0].x += t0v.x; A[0].y += t0v.y;
  A[TS].x += t1v.x; A[TS].y += t1v.y;
  A[2 * TS].x += t2v.x; A[2 * TS].y += t2v.y;
  A[3 * TS].x += t3v.x; A[3 * TS].y += t3v.y;
  const double gx = A[0].x + A[TS].x + A[2 * TS].x + A[3 * TS].x;
  const double gy = A[0].y + A[TS].y + A[2 * TS].y + A[3 * TS].y;
  g[long(t) * NR + r] = mk<R>(R(gx), R(gy));
}

// Energy partials: e[(j)*4 + slot] = sum_r conj(psi_j) acc_slot,t / N^3 (deterministic tree, one block per (t, slot))
template <typename R, int N>
__global__ void __launch_bounds__(256) k_epart(const cx<R>* psi, const cx<double>* acc, int t0, int T, double* e) {
  constexpr long NR = long(N) * N * N;
  const int t = blockIdx.x / 4, slot = blockIdx.x % 4;
  const cx<R>* p = psi + long(t0 + t) * NR;
  const cx<double>* a = acc + (long(slot) * T + t) * NR;
  double s = 0;
  for (long r = threadIdx.x; r < NR; r += blockDim.x) {
    const double pr = p[r].x, pi = p[r].y;
    s += pr * a[r].x + pi * a[r].y;   // Re(conj(psi) acc)
  }
  __shared__ double red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (int(threadIdx.x) < h) red[threadIdx.x] += red[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) e[long(t0 + t) * 4 + slot] = red[0] / double(NR);
}

}  // namespace tcmi
