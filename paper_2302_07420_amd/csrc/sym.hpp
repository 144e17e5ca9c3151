// Crystal-symmetry expansion (Sec. 2.6.1 for the orbitals; Sec. 2.6.4, the relations of Algs. 3a2 and
// 3a4 between the fields of an irreducible k-point and those of its images).
//
// An operation {R | tau} maps fractional positions x -> R (x + tau) (R integer, acting on lattice
// coordinates; S = L^T R L^-T in Cartesian coordinates, L the lattice rows).  The orbital of k-point
// k = R^T k0 - b (b integer, k inside the mesh cell) is generated from that of its representative k0 as
//   u_k(x) = e^{2 pi i b.x} u_k0(R (x + tau)),   c_k(m) = c_k0(m0) e^{2 pi i (m - b).tau},  m = R^T m0 + b.
// Fields built from the orbitals then follow with the same operation:
//   h5_k(x) = h5_k0(R (x + tau))                                   (scalar, Alg. 3a2),
//   H3_k(x) = e^{2 pi i b.x} S^T H3_k0(R (x + tau))                (Cartesian vector, Alg. 3a4),
//   (H c)_k(m) = (H c)_k0(m0) e^{2 pi i (m - b).tau}               (the operator's output).
// On an N^3 grid with N tau integer the map x -> R (x + tau) permutes the grid points.
#pragma once

namespace tcmi {

struct SymK {
  int rk;         // index of the representative among the representatives (0 .. nirr - 1)
  int R[9];       // row-major, x -> R x in lattice coordinates
  int v[3];       // R (N tau), the grid offset of the operation
  int b[3];       // R^T k0 - k
  double St[9];   // S^T, row-major, Cartesian
};

// h5[a], H3[a] for every orbital a = k nb + mu from the representatives' rows (a0 = rk nb + mu):
// h5I [nirr nb][N^3] (real), H3I [nirr nb][3][N^3], outputs [P][N^3] and [P][3][N^3].
template <typename R, int N>
__global__ void k_sym_fields(const SymK* sk, int nb, int P, const R* h5I, const cx<R>* H3I, R* h5, cx<R>* H3) {
  constexpr long NR = long(N) * N * N;
  const long id = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id >= long(P) * NR) return;
  const int a = int(id / NR);
  const long r = id - long(a) * NR;
  const SymK& s = sk[a / nb];
  const long a0 = long(s.rk) * nb + a % nb;
  const int n[3] = {int(r % N), int((r / N) % N), int(r / (long(N) * N))};
  int m[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const int t = s.R[3 * i] * n[0] + s.R[3 * i + 1] * n[1] + s.R[3 * i + 2] * n[2] + s.v[i];
    m[i] = ((t % N) + N) % N;
  }
  const long r0 = (long(m[2]) * N + m[1]) * N + m[0];
  h5[id] = h5I[a0 * NR + r0];
  // e^{2 pi i b.n / N}, with b.n reduced modulo N first
  const int bn = (((s.b[0] * n[0] + s.b[1] * n[1] + s.b[2] * n[2]) % N) + N) % N;
  double sn, cs;
  sincospi(2.0 * double(bn) / double(N), &sn, &cs);
  cx<double> v[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const cx<R> x = H3I[(a0 * 3 + d) * NR + r0];
    v[d] = mk<double>(double(x.x), double(x.y));
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double re = 0, im = 0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      re += s.St[3 * c + d] * v[d].x;
      im += s.St[3 * c + d] * v[d].y;
    }
    H3[(long(a) * 3 + c) * NR + r] = mk<R>(R(re * cs - im * sn), R(re * sn + im * cs));
  }
}

// (H c) of every orbital from the representatives' outputs: out[k][mu][g] = ph[k][g] outI[rk][mu][g0[k][g]]
// (complex128, [.][.][npw_max]; zero beyond npw(k)).
__global__ void k_sym_coef(const SymK* sk, const int* g0, const double* ph, const int* npw, int nk, int nb,
                           int npm, const double* outI, double* out) {
  const long id = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id >= long(nk) * nb * npm) return;
  const int g = int(id % npm);
  const long kb = id / npm;
  const int k = int(kb / nb), mu = int(kb % nb);
  double re = 0, im = 0;
  if (g < npw[k]) {
    const long src = (long(sk[k].rk) * nb + mu) * npm + g0[long(k) * npm + g];
    const double xr = outI[2 * src], xi = outI[2 * src + 1];
    const double pr = ph[2 * (long(k) * npm + g)], pi = ph[2 * (long(k) * npm + g) + 1];
    re = pr * xr - pi * xi;
    im = pr * xi + pi * xr;
  }
  out[2 * id] = re;
  out[2 * id + 1] = im;
}

// per-orbital energy slots of every orbital from those of its representative (they are invariant)
__global__ void k_sym_epart(const SymK* sk, int nb, int P, int nslot, const double* eI, double* e) {
  const long id = long(blockIdx.x) * blockDim.x + threadIdx.x;
  if (id >= long(P) * nslot) return;
  const int a = int(id / nslot), s = int(id % nslot);
  e[id] = eI[(long(sk[a / nb].rk) * nb + a % nb) * nslot + s];
}

}  // namespace tcmi
