// Register-resident mixed-radix Stockham FFT for one line of compile-time length N.
//
// One thread owns a whole line (N complex values in VGPRs).  The radix plan,
// every index and every twiddle index are compile-time constants after
// unrolling, so the transform is straight-line code with no LDS traffic and no
// barriers; planes and volumes are turned between axes by the calling kernels.
// Direction DIR = -1 computes X_k = sum_n x_n e^{-2 pi i nk/N} (forward), DIR = +1
// the unnormalised inverse.  Twiddles come from a table of e^{-2 pi i m/N}
// written in FP64 by the host (constant memory, scalar loads).
#pragma once
#include <hip/hip_runtime.h>

namespace tcmi {

template <typename R>
struct cx {
  R x, y;
};

template <typename R>
__host__ __device__ __forceinline__ cx<R> mk(R a, R b) { return cx<R>{a, b}; }
template <typename R>
__device__ __forceinline__ cx<R> operator+(cx<R> a, cx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ cx<R> operator-(cx<R> a, cx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ cx<R> operator*(cx<R> a, cx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R>
__device__ __forceinline__ cx<R> operator*(R s, cx<R> a) { return {s * a.x, s * a.y}; }
template <typename R>
__device__ __forceinline__ cx<R> conjg(cx<R> a) { return {a.x, -a.y}; }
template <typename R>
__device__ __forceinline__ cx<R> mul_i(cx<R> a) { return {-a.y, a.x}; }        // i a
template <typename R>
__device__ __forceinline__ cx<R> cmulc(cx<R> a, cx<R> b) {                      // conj(a) b
  return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}

// twiddle tables (filled by the host): offsets per supported length
constexpr int kTwOff8 = 0, kTwOff12 = 8, kTwOff16 = 20, kTwOff24 = 36, kTwOff32 = 60, kTwOff48 = 92,
              kTwTotal = 140;
constexpr int tw_off(int N) {
  return N == 8 ? kTwOff8 : N == 12 ? kTwOff12 : N == 16 ? kTwOff16 : N == 24 ? kTwOff24
       : N == 32 ? kTwOff32 : N == 48 ? kTwOff48 : -1;
}

// defined here: this header is compiled into exactly one translation unit
__constant__ double c_tw64[2 * kTwTotal];
__constant__ float c_tw32[2 * kTwTotal];

template <typename R>
__device__ __forceinline__ cx<R> tw_load(int idx);
template <>
__device__ __forceinline__ cx<double> tw_load<double>(int idx) { return {c_tw64[2 * idx], c_tw64[2 * idx + 1]}; }
template <>
__device__ __forceinline__ cx<float> tw_load<float>(int idx) { return {c_tw32[2 * idx], c_tw32[2 * idx + 1]}; }

// e^{DIR 2 pi i a / N}
template <typename R, int N, int DIR>
__device__ __forceinline__ cx<R> twiddle(int a) {
  cx<R> w = tw_load<R>(tw_off(N) + a);   // e^{-2 pi i a/N}
  return DIR < 0 ? w : conjg(w);
}

// v e^{DIR 2 pi i a / N}.  The index is a constant after unrolling: multiples of N/4 become sign
// swaps and odd multiples of N/8 two additions and two multiplications; the rest use the table.
template <typename R, int N, int DIR>
__device__ __forceinline__ cx<R> twiddle_mul(cx<R> v, int a) {
  a %= N;
  if (a == 0) return v;
  if (2 * a == N) return {-v.x, -v.y};
  if (4 * a == N) return DIR < 0 ? cx<R>{v.y, -v.x} : cx<R>{-v.y, v.x};        // -i v : i v
  if (4 * a == 3 * N) return DIR < 0 ? cx<R>{-v.y, v.x} : cx<R>{v.y, -v.x};    //  i v : -i v
  if (N % 8 == 0 && (8 * a) % N == 0) {
    // e^{DIR i pi t/4}, t odd: (c, s) with |c| = |s| = sqrt(1/2)
    const int t = 8 * a / N;
    const R h = R(0.70710678118654752440);
    const R c = (t == 1 || t == 7) ? h : -h;
    const R sn = R(DIR) * ((t == 1 || t == 3) ? h : -h);
    if (c == sn) return {c * (v.x - v.y), c * (v.x + v.y)};
    return {c * (v.x + v.y), c * (v.y - v.x)};
  }
  return v * twiddle<R, N, DIR>(a);
}

template <typename R, int DIR>
__device__ __forceinline__ void dft2(cx<R>* v) {
  cx<R> a = v[0], b = v[1];
  v[0] = a + b;
  v[1] = a - b;
}

template <typename R, int DIR>
__device__ __forceinline__ void dft3(cx<R>* v) {
  const R h = R(0.86602540378443864676);   // sqrt(3)/2
  cx<R> a = v[0], b = v[1], c = v[2];
  cx<R> t1 = b + c;
  cx<R> t2 = a - R(0.5) * t1;
  cx<R> d = b - c;
  cx<R> t3 = mul_i(R(DIR) * h * d);      // i DIR (sqrt3/2) (b - c)
  v[0] = a + t1;
  v[1] = t2 + t3;
  v[2] = t2 - t3;
}

template <typename R, int DIR>
__device__ __forceinline__ void dft4(cx<R>* v) {
  cx<R> a = v[0], b = v[1], c = v[2], d = v[3];
  cx<R> s0 = a + c, s1 = a - c, s2 = b + d, s3 = b - d;
  cx<R> js3 = mul_i(R(DIR) * s3);        // DIR i (b - d)
  v[0] = s0 + s2;
  v[1] = s1 + js3;
  v[2] = s0 - s2;
  v[3] = s1 - js3;
}

template <typename R, int DIR, int RAD>
__device__ __forceinline__ void dft(cx<R>* v) {
  if constexpr (RAD == 2) dft2<R, DIR>(v);
  else if constexpr (RAD == 3) dft3<R, DIR>(v);
  else dft4<R, DIR>(v);
}

// One Stockham stage: butterflies of radix RAD after sub-transforms of length NS.
template <typename R, int N, int DIR, int NS, int RAD>
__device__ __forceinline__ void stage(cx<R>* x) {
  cx<R> y[N];
#pragma unroll
  for (int j = 0; j < N / RAD; ++j) {
    const int k = j % NS;
    cx<R> v[RAD];
#pragma unroll
    for (int m = 0; m < RAD; ++m) {
      v[m] = x[j + m * (N / RAD)];
      if (m * k != 0) v[m] = twiddle_mul<R, N, DIR>(v[m], m * k * (N / (NS * RAD)));
    }
    dft<R, DIR, RAD>(v);
#pragma unroll
    for (int p = 0; p < RAD; ++p) y[(j / NS) * NS * RAD + k + p * NS] = v[p];
  }
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] = y[i];
}

template <typename R, int N, int DIR, int NS, int RAD, int... REST>
__device__ __forceinline__ void stages(cx<R>* x) {
  stage<R, N, DIR, NS, RAD>(x);
  if constexpr (sizeof...(REST) > 0) stages<R, N, DIR, NS * RAD, REST...>(x);
}

// Power-of-two lengths: Stockham stages (radix 4, then 2 or 4).
template <typename R, int N, int DIR>
__device__ __forceinline__ void fft_pow2(cx<R>* x) {
  if constexpr (N == 4) dft4<R, DIR>(x);
  else if constexpr (N == 8) stages<R, 8, DIR, 1, 4, 2>(x);
  else if constexpr (N == 16) stages<R, 16, DIR, 1, 4, 4>(x);
  else stages<R, 32, DIR, 1, 4, 4, 2>(x);
}

// Lengths 3 M (M = 4, 8, 16, coprime to 3): Good-Thomas prime-factor algorithm, no twiddles between
// the two factors.  Input n = (M n1 + 3 n2) mod N goes to a[n1][n2]; M-point transforms along n2,
// 3-point transforms along n1; output (k1, k2) is X[(M U k1 + 3 V k2) mod N] with U = M^-1 mod 3 and
// V = 3^-1 mod M (Chinese remainder map).  All indices are compile-time constants after unrolling.
template <typename R, int M, int DIR>
__device__ __forceinline__ void fft_pfa3(cx<R>* x) {
  constexpr int N = 3 * M;
  constexpr int U = (M % 3 == 1) ? 1 : 2;
  constexpr int V = (M == 4) ? 3 : (M == 8) ? 3 : 11;
  static_assert((M * U) % 3 == 1 && (3 * V) % M == 1, "inverse residues");
  cx<R> a[3][M];
#pragma unroll
  for (int n1 = 0; n1 < 3; ++n1) {
#pragma unroll
    for (int n2 = 0; n2 < M; ++n2) a[n1][n2] = x[(M * n1 + 3 * n2) % N];
    fft_pow2<R, M, DIR>(a[n1]);
  }
#pragma unroll
  for (int k2 = 0; k2 < M; ++k2) {
    cx<R> t[3] = {a[0][k2], a[1][k2], a[2][k2]};
    dft3<R, DIR>(t);
#pragma unroll
    for (int k1 = 0; k1 < 3; ++k1) x[(M * U * k1 + 3 * V * k2) % N] = t[k1];
  }
}

template <typename R, int N, int DIR>
__device__ __forceinline__ void fft_line(cx<R>* x) {
  static_assert(N == 8 || N == 12 || N == 16 || N == 24 || N == 32 || N == 48, "unsupported length");
  if constexpr (N == 12 || N == 24 || N == 48) fft_pfa3<R, N / 3, DIR>(x);
  else fft_pow2<R, N, DIR>(x);
}

}  // namespace tcmi
