// Eigenvalues and right/left eigenvectors of a small dense complex matrix (FP64), for the subspace
// step of the block-Davidson iteration (Sec. 2.4: the subspace matrix of the non-Hermitian operator
// is diagonalised).  Sequential code, callable on the host and on the device (one thread per matrix).
//
// Method (textbook): Householder reduction to upper Hessenberg form, complex Schur form by
// shifted QR iterations with Givens rotations (Wilkinson shift, exceptional shifts on stagnation,
// deflation at negligible subdiagonals), then eigenvectors of the triangular factor by back and
// forward substitution, transformed back with the accumulated unitary factor.
#pragma once
#include <hip/hip_runtime.h>

namespace tcmi {

struct zc {
  double r, i;
};
__host__ __device__ inline zc zmk(double r, double i) { return zc{r, i}; }
__host__ __device__ inline zc operator+(zc a, zc b) { return {a.r + b.r, a.i + b.i}; }
__host__ __device__ inline zc operator-(zc a, zc b) { return {a.r - b.r, a.i - b.i}; }
__host__ __device__ inline zc operator*(zc a, zc b) { return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r}; }
__host__ __device__ inline zc operator*(double s, zc a) { return {s * a.r, s * a.i}; }
__host__ __device__ inline zc zconj(zc a) { return {a.r, -a.i}; }
__host__ __device__ inline double zabs(zc a) { return hypot(a.r, a.i); }
__host__ __device__ inline double zabs1(zc a) { return fabs(a.r) + fabs(a.i); }
__host__ __device__ inline zc zdiv(zc a, zc b) {
  // Smith's algorithm
  if (fabs(b.r) >= fabs(b.i)) {
    const double t = b.i / b.r, d = b.r + b.i * t;
    return {(a.r + a.i * t) / d, (a.i - a.r * t) / d};
  }
  const double t = b.r / b.i, d = b.r * t + b.i;
  return {(a.r * t + a.i) / d, (a.i * t - a.r) / d};
}
__host__ __device__ inline zc zsqrt(zc a) {
  const double m = zabs(a);
  if (m == 0.0) return {0.0, 0.0};
  if (a.r >= 0.0) {
    const double t = sqrt(0.5 * (m + a.r));
    return {t, a.i / (2.0 * t)};
  }
  const double t = sqrt(0.5 * (m - a.r));
  return {fabs(a.i) / (2.0 * t), a.i >= 0.0 ? t : -t};
}

// Row-major m x m matrices: a[i * m + j].
//   A  (in, destroyed): the matrix; on return it holds the upper-triangular Schur factor T
//   Q  (out): unitary factor, A_in = Q T Q^H
//   w  (out): eigenvalues w[k] = T[k][k]
//   VR (out, may be null): right eigenvectors as columns, VR[i * m + k], unit 2-norm
//   VL (out, may be null): left eigenvectors as columns (VL[:,k]^H A = w[k] VL[:,k]^H), unit 2-norm
//   y  (scratch): m complex
// Returns 0, or 1 if the QR iteration did not converge within 60 m sweeps.
__host__ __device__ inline int eig_small(int m, zc* A, zc* Q, zc* w, zc* VR, zc* VL, zc* y) {
  const double eps = 2.220446049250313e-16;
  double anorm = 0;
  for (int e = 0; e < m * m; ++e) anorm = fmax(anorm, zabs1(A[e]));
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < m; ++j) Q[i * m + j] = zmk(i == j ? 1.0 : 0.0, 0.0);
  // 1. Householder reduction to Hessenberg form: for column k, reflect x = A[k+1:m, k] onto alpha e_1
  for (int k = 0; k + 2 < m; ++k) {
    double xn = 0;
    for (int i = k + 1; i < m; ++i) xn += A[i * m + k].r * A[i * m + k].r + A[i * m + k].i * A[i * m + k].i;
    xn = sqrt(xn);
    if (xn == 0.0) continue;
    const zc x0 = A[(k + 1) * m + k];
    const double a0 = zabs(x0);
    const zc ph = a0 > 0 ? zmk(x0.r / a0, x0.i / a0) : zmk(1.0, 0.0);
    const zc alpha = -xn * ph;   // alpha = -e^{i arg x0} ||x||
    // v = x - alpha e_1 (stored in y[k+1..m)), H = I - 2 v v^H / (v^H v)
    double vn = 0;
    for (int i = k + 1; i < m; ++i) {
      y[i] = A[i * m + k];
      if (i == k + 1) y[i] = y[i] - alpha;
      vn += y[i].r * y[i].r + y[i].i * y[i].i;
    }
    if (vn == 0.0) continue;
    const double beta = 2.0 / vn;
    // A <- H A (rows k+1..m, columns k..m)
    for (int j = k; j < m; ++j) {
      zc s = zmk(0, 0);
      for (int i = k + 1; i < m; ++i) s = s + zconj(y[i]) * A[i * m + j];
      s = beta * s;
      for (int i = k + 1; i < m; ++i) A[i * m + j] = A[i * m + j] - y[i] * s;
    }
    // A <- A H (all rows, columns k+1..m); Q <- Q H
    for (int i = 0; i < m; ++i) {
      zc s = zmk(0, 0), t = zmk(0, 0);
      for (int j = k + 1; j < m; ++j) {
        s = s + A[i * m + j] * y[j];
        t = t + Q[i * m + j] * y[j];
      }
      s = beta * s;
      t = beta * t;
      for (int j = k + 1; j < m; ++j) {
        A[i * m + j] = A[i * m + j] - s * zconj(y[j]);
        Q[i * m + j] = Q[i * m + j] - t * zconj(y[j]);
      }
    }
    for (int i = k + 2; i < m; ++i) A[i * m + k] = zmk(0, 0);
  }
  // 2. Shifted QR on the Hessenberg matrix, deflating from the bottom
  int ihi = m - 1, its = 0, total = 0;
  const int maxit = 60 * (m > 1 ? m : 1);
  while (ihi > 0) {
    if (total++ > maxit) return 1;
    int l = ihi;
    for (; l > 0; --l) {
      const double s = zabs1(A[(l - 1) * m + l - 1]) + zabs1(A[l * m + l]);
      const double ref = s > 0 ? s : anorm;
      if (zabs1(A[l * m + l - 1]) <= eps * ref) {
        A[l * m + l - 1] = zmk(0, 0);
        break;
      }
    }
    if (l == ihi) {   // one eigenvalue converged
      --ihi;
      its = 0;
      continue;
    }
    ++its;
    // Wilkinson shift from the trailing 2 x 2 block; exceptional shift every 10 stagnant sweeps
    zc mu;
    if (its % 10 == 0) {
      mu = A[ihi * m + ihi] + zmk(0.75 * zabs1(A[ihi * m + ihi - 1]), 0.0);
    } else {
      const zc a = A[(ihi - 1) * m + ihi - 1], b = A[(ihi - 1) * m + ihi], c = A[ihi * m + ihi - 1],
               d = A[ihi * m + ihi];
      const zc hd = 0.5 * (a - d);
      const zc disc = zsqrt(hd * hd + b * c);
      // eigenvalues of the block: (a + d)/2 +- disc; take the one closer to d
      const zc half = 0.5 * (a + d);
      const zc e1 = half + disc, e2 = half - disc;
      mu = zabs1(e1 - d) <= zabs1(e2 - d) ? e1 : e2;
    }
    // explicit shifted QR sweep on rows/columns l..ihi with Givens rotations G_k = [c s; -conj(s) c]:
    // H - mu = QR by left rotations (full rows, columns k..m), then RQ + mu by right rotations (full
    // columns, rows 0..ihi), so that A tends to the complete Schur form.  c is kept in y[k], s in w[k]
    // (w is scratch until the eigenvalues are written).
    for (int k = l; k <= ihi; ++k) A[k * m + k] = A[k * m + k] - mu;
    for (int k = l; k < ihi; ++k) {
      const zc f = A[k * m + k], g = A[(k + 1) * m + k];
      const double fa = zabs(f), ga = zabs(g);
      double c;
      zc sn;
      if (ga == 0.0) {
        c = 1.0;
        sn = zmk(0, 0);
      } else if (fa == 0.0) {
        c = 0.0;
        sn = zmk(g.r / ga, -g.i / ga);   // conj(g)/|g|
      } else {
        const double nr = hypot(fa, ga);
        c = fa / nr;
        const zc fph = zmk(f.r / fa, f.i / fa);
        sn = fph * zmk(g.r / nr, -g.i / nr);   // (f/|f|) conj(g) / r
      }
      // rows k, k+1: [c s; -conj(s) c] applied from the left, columns k..m
      for (int j = k; j < m; ++j) {
        const zc u = A[k * m + j], v = A[(k + 1) * m + j];
        A[k * m + j] = c * u + sn * v;
        A[(k + 1) * m + j] = c * v - zconj(sn) * u;
      }
      y[k] = zmk(c, 0.0);
      w[k] = sn;
      A[(k + 1) * m + k] = zmk(0, 0);
    }
    // right rotations: columns k, k+1 times G_k^H
    for (int k = l; k < ihi; ++k) {
      const double c = y[k].r;
      const zc sn = w[k];
      for (int i = 0; i <= ihi; ++i) {
        const zc u = A[i * m + k], v = A[i * m + k + 1];
        A[i * m + k] = c * u + zconj(sn) * v;
        A[i * m + k + 1] = c * v - sn * u;
      }
      for (int i = 0; i < m; ++i) {
        const zc u = Q[i * m + k], v = Q[i * m + k + 1];
        Q[i * m + k] = c * u + zconj(sn) * v;
        Q[i * m + k + 1] = c * v - sn * u;
      }
    }
    for (int k = l; k <= ihi; ++k) A[k * m + k] = A[k * m + k] + mu;
  }
  for (int k = 0; k < m; ++k) w[k] = A[k * m + k];
  const double small = eps * (anorm > 0 ? anorm : 1.0);
  // 3. right eigenvectors: T z = w_k z with z_k = 1, z_j = 0 (j > k), back substitution for j < k
  if (VR) {
    for (int k = 0; k < m; ++k) {
      for (int j = 0; j < m; ++j) y[j] = zmk(j == k ? 1.0 : 0.0, 0.0);
      for (int j = k - 1; j >= 0; --j) {
        zc s = zmk(0, 0);
        for (int i = j + 1; i <= k; ++i) s = s + A[j * m + i] * y[i];
        zc d = A[j * m + j] - w[k];
        if (zabs1(d) < small) d = zmk(small, 0.0);
        y[j] = zdiv(zmk(0, 0) - s, d);
      }
      double nrm = 0;
      for (int i = 0; i < m; ++i) {
        zc s = zmk(0, 0);
        for (int j = 0; j <= k; ++j) s = s + Q[i * m + j] * y[j];
        VR[i * m + k] = s;
        nrm += s.r * s.r + s.i * s.i;
      }
      nrm = 1.0 / sqrt(nrm);
      for (int i = 0; i < m; ++i) VR[i * m + k] = nrm * VR[i * m + k];
    }
  }
  // 4. left eigenvectors: u^T T = w_k u^T with u_k = 1, u_j = 0 (j < k), forward substitution for
  //    j > k; the left eigenvector of A is Q conj(u)
  if (VL) {
    for (int k = 0; k < m; ++k) {
      for (int j = 0; j < m; ++j) y[j] = zmk(j == k ? 1.0 : 0.0, 0.0);
      for (int j = k + 1; j < m; ++j) {
        zc s = zmk(0, 0);
        for (int i = k; i < j; ++i) s = s + y[i] * A[i * m + j];
        zc d = w[k] - A[j * m + j];
        if (zabs1(d) < small) d = zmk(small, 0.0);
        y[j] = zdiv(s, d);
      }
      double nrm = 0;
      for (int i = 0; i < m; ++i) {
        zc s = zmk(0, 0);
        for (int j = k; j < m; ++j) s = s + Q[i * m + j] * zconj(y[j]);
        VL[i * m + k] = s;
        nrm += s.r * s.r + s.i * s.i;
      }
      nrm = 1.0 / sqrt(nrm);
      for (int i = 0; i < m; ++i) VL[i * m + k] = nrm * VL[i * m + k];
    }
  }
  return 0;
}

}  // namespace tcmi
