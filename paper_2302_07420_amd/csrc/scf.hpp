// Device kernels of the block-Davidson self-consistent loop (Sec. 2.4), FP64, coefficient space.
//
// Subspace layout: block-major, V[(p * nk + k) * nb + i][npw_max] complex128 for block p (0..pmax),
// k-point k, band i; column j = p nb + i of the subspace of k-point k.  The same layout holds h V.
#pragma once
#include "eig_small.hpp"
#include "reduce.hpp"

namespace tcmi {

__device__ __forceinline__ long sub_row(int p, int k, int i, int nk, int nb) { return (long(p) * nk + k) * nb + i; }

// Gram-Schmidt of columns j0..j1-1 of each k-point's subspace against all earlier valid columns (and
// each other, in order), classical with one re-orthogonalisation pass.  A column whose norm is below atol
// before the projection, or below rtol times that norm after it (linearly dependent), is zeroed and
// marked invalid (Sec. 2.4 drops such trial vectors).  One block per k.
__global__ void __launch_bounds__(256) k_gram_schmidt(double* V, int* valid, const int* npw, int nk, int nb,
                                                     int npw_max, int mcols, int j0, int j1, double atol,
                                                     double rtol) {
  const int k = blockIdx.x;
  const int n = npw[k];
  for (int j = j0; j < j1; ++j) {
    double* vj = V + 2 * sub_row(j / nb, k, j % nb, nk, nb) * npw_max;
    double n0r = 0, n0i = 0;
    for (int g = threadIdx.x; g < n; g += blockDim.x) n0r += vj[2 * g] * vj[2 * g] + vj[2 * g + 1] * vj[2 * g + 1];
    wg_sum2(n0r, n0i);
    const double norm0 = sqrt(n0r);
    for (int pass = 0; pass < 2; ++pass)
      for (int i = 0; i < j; ++i) {
        if (!valid[k * mcols + i]) continue;
        const double* vi = V + 2 * sub_row(i / nb, k, i % nb, nk, nb) * npw_max;
        double cr = 0, ci = 0;   // <v_i|v_j>
        for (int g = threadIdx.x; g < n; g += blockDim.x) {
          cr += vi[2 * g] * vj[2 * g] + vi[2 * g + 1] * vj[2 * g + 1];
          ci += vi[2 * g] * vj[2 * g + 1] - vi[2 * g + 1] * vj[2 * g];
        }
        wg_sum2(cr, ci);
        for (int g = threadIdx.x; g < n; g += blockDim.x) {
          const double xr = vi[2 * g], xi = vi[2 * g + 1];
          vj[2 * g] -= cr * xr - ci * xi;
          vj[2 * g + 1] -= cr * xi + ci * xr;
        }
        __syncthreads();
      }
    double nr = 0, ni = 0;
    for (int g = threadIdx.x; g < n; g += blockDim.x) nr += vj[2 * g] * vj[2 * g] + vj[2 * g + 1] * vj[2 * g + 1];
    wg_sum2(nr, ni);
    const double nrm = sqrt(nr);
    const bool ok = norm0 >= atol && nrm > rtol * norm0 && nrm > 1e-300;
    const double sc = ok ? 1.0 / nrm : 0.0;
    for (int g = threadIdx.x; g < npw_max; g += blockDim.x) {
      vj[2 * g] = g < n ? vj[2 * g] * sc : 0.0;
      vj[2 * g + 1] = g < n ? vj[2 * g + 1] * sc : 0.0;
    }
    if (threadIdx.x == 0) valid[k * mcols + j] = ok ? 1 : 0;
    __syncthreads();
  }
}

// h v += |k+G|^2/2 v for the nb rows of block p of every k-point (one thread per element)
__global__ void k_add_kinetic(const double* V, double* HV, const double* kg, const int* npw, int nk, int nb,
                              int npw_max, int p) {
  const long id = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id >= long(nk) * nb * npw_max) return;
  const long row = id / npw_max;
  const int g = int(id - row * npw_max), k = int(row / nb);
  if (g >= npw[k]) return;
  const double* q = kg + (long(k) * npw_max + g) * 3;
  const double e = 0.5 * (q[0] * q[0] + q[1] * q[1] + q[2] * q[2]);
  const long o = 2 * ((long(p) * nk * nb + row) * npw_max + g);
  HV[o] += e * V[o];
  HV[o + 1] += e * V[o + 1];
}

// eps[k][i] = <v_i|h v_i> for the first block (Rayleigh quotients; one block per (k, i))
__global__ void __launch_bounds__(256) k_rayleigh(const double* V, const double* HV, const int* npw, int nk, int nb,
                                                 int npw_max, double* eps) {
  const int k = blockIdx.x / nb, i = blockIdx.x % nb;
  const double* v = V + 2 * sub_row(0, k, i, nk, nb) * npw_max;
  const double* h = HV + 2 * sub_row(0, k, i, nk, nb) * npw_max;
  double sr = 0, si = 0;
  for (int g = threadIdx.x; g < npw[k]; g += blockDim.x) {
    sr += v[2 * g] * h[2 * g] + v[2 * g + 1] * h[2 * g + 1];
    si += v[2 * g] * h[2 * g + 1] - v[2 * g + 1] * h[2 * g];
  }
  wg_sum2(sr, si);
  if (threadIdx.x == 0) {
    eps[2 * (k * nb + i)] = sr;
    eps[2 * (k * nb + i) + 1] = si;
  }
}

// Block p of the expansion: v_{p nb + i} = P (h - eps_i) v_{(p-1) nb + i}, with the preconditioner of
// Payne et al. as a function of x = (|k+G|^2/2) / T_i, T_i = sum_G |k+G|^2/2 |v~(G)|^2 of the vector the
// residual is taken of (one block per (k, i)).  A residual whose norm before preconditioning is below
// atol is written as zero (the trial vector is dropped): the preconditioner can shrink a residual by
// orders of magnitude when T_i is small, so the size test is made before it.
__global__ void __launch_bounds__(256) k_precond_residual(double* V, const double* HV, const double* eps,
                                                         const double* kg, const int* npw, int nk, int nb,
                                                         int npw_max, int p, double atol) {
  const int k = blockIdx.x / nb, i = blockIdx.x % nb;
  const double* v = V + 2 * sub_row(p - 1, k, i, nk, nb) * npw_max;
  const double* h = HV + 2 * sub_row(p - 1, k, i, nk, nb) * npw_max;
  double* out = V + 2 * sub_row(p, k, i, nk, nb) * npw_max;
  const double* q0 = kg + long(k) * npw_max * 3;
  const double er = eps[2 * (k * nb + i)], ei = eps[2 * (k * nb + i) + 1];
  double t = 0, rn = 0;
  for (int g = threadIdx.x; g < npw[k]; g += blockDim.x) {
    const double* q = q0 + 3 * g;
    t += 0.5 * (q[0] * q[0] + q[1] * q[1] + q[2] * q[2]) * (v[2 * g] * v[2 * g] + v[2 * g + 1] * v[2 * g + 1]);
    const double rr = h[2 * g] - (er * v[2 * g] - ei * v[2 * g + 1]);
    const double ri = h[2 * g + 1] - (er * v[2 * g + 1] + ei * v[2 * g]);
    rn += rr * rr + ri * ri;
  }
  wg_sum2(t, rn);
  const bool keep = sqrt(rn) >= atol;
  for (int g = threadIdx.x; g < npw_max; g += blockDim.x) {
    double rr = 0, ri = 0;
    if (keep && g < npw[k]) {
      const double* q = q0 + 3 * g;
      const double x = t > 0 ? 0.5 * (q[0] * q[0] + q[1] * q[1] + q[2] * q[2]) / t : 0.0;
      const double num = 27.0 + x * (18.0 + x * (12.0 + 8.0 * x));
      const double pre = num / (num + 16.0 * x * x * x * x);
      rr = pre * (h[2 * g] - (er * v[2 * g] - ei * v[2 * g + 1]));
      ri = pre * (h[2 * g + 1] - (er * v[2 * g + 1] + ei * v[2 * g]));
    }
    out[2 * g] = rr;
    out[2 * g + 1] = ri;
  }
}

// Subspace matrix Hs[k][a][b] = <v_a|h v_b> over the first mcols columns (one block per (k, a, b))
__global__ void __launch_bounds__(256) k_subspace_matrix(const double* V, const double* HV, const int* npw, int nk,
                                                        int nb, int npw_max, int mcols, double* Hs) {
  const int id = blockIdx.x;
  const int k = id / (mcols * mcols), a = (id / mcols) % mcols, b = id % mcols;
  const double* x = V + 2 * sub_row(a / nb, k, a % nb, nk, nb) * npw_max;
  const double* y = HV + 2 * sub_row(b / nb, k, b % nb, nk, nb) * npw_max;
  double sr = 0, si = 0;
  for (int g = threadIdx.x; g < npw[k]; g += blockDim.x) {
    sr += x[2 * g] * y[2 * g] + x[2 * g + 1] * y[2 * g + 1];
    si += x[2 * g] * y[2 * g + 1] - x[2 * g + 1] * y[2 * g];
  }
  wg_sum2(sr, si);
  if (threadIdx.x == 0) {
    Hs[2 * id] = sr;
    Hs[2 * id + 1] = si;
  }
}

// Per k-point (one thread): restrict Hs to the valid columns, diagonalise, order the eigenvalues by
// real part and write the nb lowest with their right (X) and left (Y) eigenvectors, expanded over all
// mcols columns (zero at invalid ones): X[k][j][i] is the coefficient of column j in eigenvector i.
// work: per k, 4 M^2 + 2 M complex; M <= 512.  status[k] = 0, 1 (no convergence) or 2 (fewer valid columns than nb).
// change[k] = largest norm, over the selected eigenvectors, of the part outside the first nb columns (the
// previous orbitals): the orbitals' move out of their previous span (the basis is orthonormal).
__global__ void k_subspace_eig(const double* Hs, const int* valid, int nk, int nb, int mcols, double* work,
                               double* X, double* Y, double* evals, int* status, double* change) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= nk) return;
  const int M = mcols;
  zc* wk = reinterpret_cast<zc*>(work) + long(k) * (4L * M * M + 2L * M);
  zc* A = wk;
  zc* Q = A + M * M;
  zc* VR = Q + M * M;
  zc* VL = VR + M * M;
  zc* w = VL + M * M;
  zc* y = w + M;
  const zc* H = reinterpret_cast<const zc*>(Hs) + long(k) * M * M;
  int cols[512];
  int m = 0;
  for (int j = 0; j < M && m < 512; ++j)
    if (valid[k * M + j]) cols[m++] = j;
  zc* Xk = reinterpret_cast<zc*>(X) + long(k) * M * nb;
  zc* Yk = reinterpret_cast<zc*>(Y) + long(k) * M * nb;
  for (int e = 0; e < M * nb; ++e) Xk[e] = Yk[e] = zmk(0, 0);
  if (m < nb) {
    status[k] = 2;
    return;
  }
  for (int a = 0; a < m; ++a)
    for (int b = 0; b < m; ++b) A[a * m + b] = H[cols[a] * M + cols[b]];
  const int st = eig_small(m, A, Q, w, VR, VL, y);
  status[k] = st;
  if (st != 0) return;
  // selection of the nb lowest real parts (stable: ties keep the solver's order)
  bool used[512];
  for (int a = 0; a < m; ++a) used[a] = false;
  zc* ev = reinterpret_cast<zc*>(evals) + long(k) * nb;
  double chg = 0;
  for (int i = 0; i < nb; ++i) {
    int best = -1;
    for (int a = 0; a < m; ++a)
      if (!used[a] && (best < 0 || w[a].r < w[best].r)) best = a;
    used[best] = true;
    ev[i] = w[best];
    double out = 0;
    for (int a = 0; a < m; ++a) {
      Xk[cols[a] * nb + i] = VR[a * m + best];
      Yk[cols[a] * nb + i] = VL[a * m + best];
      if (cols[a] >= nb) out += VR[a * m + best].r * VR[a * m + best].r + VR[a * m + best].i * VR[a * m + best].i;
    }
    chg = fmax(chg, sqrt(out));
  }
  change[k] = chg;
}

// out[k][i] = sum_j C[k][j][i] v_j (new orbitals from the subspace; one thread per element)
__global__ void k_subspace_combine(const double* V, const double* C, int nk, int nb, int npw_max, int mcols,
                                   double* out) {
  const long id = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id >= long(nk) * nb * npw_max) return;
  const long row = id / npw_max;
  const int g = int(id - row * npw_max), k = int(row / nb), i = int(row % nb);
  double sr = 0, si = 0;
  for (int j = 0; j < mcols; ++j) {
    const double* c = C + 2 * ((long(k) * mcols + j) * nb + i);
    const double* v = V + 2 * (sub_row(j / nb, k, j % nb, nk, nb) * npw_max + g);
    sr += c[0] * v[0] - c[1] * v[1];
    si += c[0] * v[1] + c[1] * v[0];
  }
  out[2 * id] = sr;
  out[2 * id + 1] = si;
}

}  // namespace tcmi
