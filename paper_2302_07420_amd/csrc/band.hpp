// Grid pieces of the divergence corrections of band (zero-weight) k-points (the band forms of Sec. 2.6:
// Eqs. divcorr_3a3, div_corr_3b3_2, div_corr_3b4_2/4, div_corr_3a4_2, 3b5_div_2, 3b6_div_band2/3).  The
// FP64 combination with the band orbitals' overlaps is done on the host.  Band targets are numbered
// j = b nb + mu (band k-point b, orbital mu); fields are per target [j][...][N^3].
#pragma once

namespace tcmi {

// h4 of the targets t0 .. t0 + nt (Cartesian, [t][3][N^3]) += V_b sum_mu a[j][mu] psiT[b nb + mu], the
// correction of the q1 sum of Alg. 3a3 (= h3 of Alg. 3b4) at q1 -> k: a = -i 4 pi A f_mu S_mu,j / Omega.
template <typename R, int N>
__global__ void k_band_dh4(const cx<R>* psiT, const double* a, const double* V, int t0, int nt, int nb, cx<R>* h4) {
  constexpr long NR = long(N) * N * N;
  const long id = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id >= long(nt) * NR) return;
  const int t = int(id / NR);
  const long r = id - long(t) * NR;
  const int j = t0 + t, b = j / nb;
  double sr = 0, si = 0;
  for (int mu = 0; mu < nb; ++mu) {
    const double ar = a[2 * (long(j) * nb + mu)], ai = a[2 * (long(j) * nb + mu) + 1];
    const cx<R> x = psiT[(long(b) * nb + mu) * NR + r];
    sr += ar * double(x.x) - ai * double(x.y);
    si += ar * double(x.y) + ai * double(x.x);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    cx<R>& h = h4[(long(t) * 3 + c) * NR + r];
    h.x += R(V[3 * b + c] * sr);
    h.y += R(V[3 * b + c] * si);
  }
}

// Band-pair grid means (one work-group of 256 per output):
//   out[((j) nb + mu) nc + c] = (1/N^3) sum_r conj(A_(b nb + mu), c) B_(j), c [F_c]
// for targets j in [j0, j0 + nj), b = j / nb; A rows b nb + mu with stride sA per row and sAc per
// component; B row (j - jB0) with strides sB, sBc; F (may be null) with component stride sFc.
template <typename TA, typename TB, typename TF>
__global__ void __launch_bounds__(256) k_band_dot(const cx<TA>* A, long sA, long sAc, const cx<TB>* B, long sB,
                                                  long sBc, int jB0, const cx<TF>* F, long sFc, int j0, int nb,
                                                  int nc, long NR, double* out) {
  const int o = blockIdx.x;
  const int c = o % nc, mu = (o / nc) % nb, j = j0 + o / (nc * nb);
  const int b = j / nb;
  const cx<TA>* a = A + (long(b) * nb + mu) * sA + c * sAc;
  const cx<TB>* bb = B + long(j - jB0) * sB + c * sBc;
  const cx<TF>* f = F ? F + c * sFc : nullptr;
  double sr = 0, si = 0;
  for (long r = threadIdx.x; r < NR; r += blockDim.x) {
    const double ar = double(a[r].x), ai = -double(a[r].y);
    double br = double(bb[r].x), bi = double(bb[r].y);
    if (f) {
      const double fr = double(f[r].x), fi = double(f[r].y);
      const double tr = br * fr - bi * fi;
      bi = br * fi + bi * fr;
      br = tr;
    }
    sr += ar * br - ai * bi;
    si += ar * bi + ai * br;
  }
  wg_sum2(sr, si);
  if (threadIdx.x == 0) {
    const long idx = (long(o / (nc * nb)) + j0) * nb * nc + long(mu) * nc + c;
    out[2 * idx] = sr / double(NR);
    out[2 * idx + 1] = si / double(NR);
  }
}

// out[j] = V_b . H3[j] (scalar fields of the band rows' h3, for the image of Eq. div_corr_3a4_2)
template <typename R, int N>
__global__ void k_band_vdot(const cx<R>* H3, const double* V, int nj, int nb, cx<R>* out) {
  constexpr long NR = long(N) * N * N;
  const long id = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id >= long(nj) * NR) return;
  const int j = int(id / NR);
  const long r = id - long(j) * NR;
  const double* v = V + 3 * (j / nb);
  double sr = 0, si = 0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const cx<R> x = H3[(long(j) * 3 + c) * NR + r];
    sr += v[c] * double(x.x);
    si += v[c] * double(x.y);
  }
  out[id] = mk<R>(R(sr), R(si));
}

// 3b6 band field of band k-point b in G space: sum_ch -2 pi A_ch (V_b . G) u~_ch(G) n~(G) (Eq. 3b6_div_band2)
template <int N>
__global__ void k_band_f3b6(const Recip rc, const double* u0, const double* u1, double c0, double c1, const double* V,
                            const cx<double>* nG, cx<double>* out) {
  constexpr long NR = long(N) * N * N;
  const long r = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (r >= NR) return;
  const int x = int(r % N), y = int((r / N) % N), z = int(r / (long(N) * N));
  const int m1 = x < N / 2 ? x : x - N, m2 = y < N / 2 ? y : y - N, m3 = z < N / 2 ? z : z - N;
  double vg = 0;
#pragma unroll
  for (int c = 0; c < 3; ++c) vg += V[c] * (m1 * rc.b[c] + m2 * rc.b[3 + c] + m3 * rc.b[6 + c]);
  out[r] = (vg * (c0 * u0[r] + c1 * u1[r])) * nG[r];
}

// pointwise products out[j] = F * psi[j] (FP64, one field F)
template <int N>
__global__ void k_band_mul(const cx<double>* F, const cx<double>* psi, int nj, cx<double>* out) {
  constexpr long NR = long(N) * N * N;
  const long id = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id >= long(nj) * NR) return;
  out[id] = F[id % NR] * psi[id];
}

}  // namespace tcmi
