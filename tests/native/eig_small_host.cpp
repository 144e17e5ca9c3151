// Host build of the small eigensolver for the CPU tests (ctypes entry point).
#include "../../paper_2302_07420_amd/csrc/eig_small.hpp"

extern "C" int eig_small_host(int m, double* a, double* w, double* vr, double* vl) {
  using tcmi::zc;
  zc* A = reinterpret_cast<zc*>(a);
  zc* Q = new zc[size_t(m) * m];
  zc* y = new zc[size_t(m)];
  const int st = tcmi::eig_small(m, A, Q, reinterpret_cast<zc*>(w), reinterpret_cast<zc*>(vr),
                                 reinterpret_cast<zc*>(vl), y);
  delete[] Q;
  delete[] y;
  return st;
}
