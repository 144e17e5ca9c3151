// Host checks of the C-ABI library under AddressSanitizer and UndefinedBehaviorSanitizer (host code
// only; built and run by tests/test_host_sanitizers.py, no device needed).
//
// The library's translation unit is compiled into this program (with TCMI_HOST_CHECK_BUILD, which keeps
// the device code to the 8-point engine so that it compiles quickly).  The program makes a context by
// hand, since tc_create needs a device, and drives the entry points that only describe the problem:
// their argument checks, and a complete description (cell, k-mesh, grid, plane-wave sets, Jastrow,
// options, symmetry, band k-points).  It also evaluates the host tables the application is built from.
// Results go to stdout, one record per line, for the test to compare with the oracle:
//   code <name> <status>                       status of a call with the named bad (or good) arguments
//   gb <sigma_aux> <delta_gb>                  Gygi-Baldereschi sum and constant (Eq. correction2)
//   jk <Q2> <A> <C> <u> <lap u> <(grad u)^2>   Jastrow kernels at |Q|^2 (Sec. 2.6.3, App. B)
//   tangent <dir> <exact> <central difference> derivative of the kernels along one parameter
//   sym <nirr> <orbit sizes...>                 representative k-points of the mesh under the operations
//   tri <pairs> <mismatches>                   triangular pair store: row offsets and the z stage's decode
//                                              of a batch's pairs, against plain enumeration
//   FAIL <line> <condition>                    an internal check that did not hold
// Input (argv[1], whitespace separated): lattice rows (9); k-mesh (3); A (2); C (2); alpha; ecut;
// nsym and nsym x (R row-major, 9 integers; tau, 3 fractions); nq and nq values of |Q|^2;
// nkb and nkb fractional band k-points.
#include "../../paper_2302_07420_amd/csrc/engine.hip"

#include <cstdio>
#include <fstream>

namespace {

int g_fail = 0;
#define EXPECT(cond)                                              \
  do {                                                            \
    if (!(cond)) {                                                \
      std::printf("FAIL %d %s\n", __LINE__, #cond);                \
      ++g_fail;                                                   \
    }                                                             \
  } while (0)

void code(const char* name, int st) { std::printf("code %s %d\n", name, st); }

// Plane waves with |k + G|^2 / 2 <= ecut that fit a grid of N points per axis.
std::vector<int32_t> sphere(const Problem& pb, int ik, double ecut) {
  double f[3];
  pb.kfrac(ik, f);
  std::vector<int32_t> m;
  const int h = pb.N / 2 - 1;
  for (int a = -h; a <= h; ++a)
    for (int b = -h; b <= h; ++b)
      for (int d = -h; d <= h; ++d) {
        double q[3];
        for (int c = 0; c < 3; ++c) q[c] = (a + f[0]) * pb.B[c] + (b + f[1]) * pb.B[3 + c] + (d + f[2]) * pb.B[6 + c];
        if (0.5 * (q[0] * q[0] + q[1] * q[1] + q[2] * q[2]) <= ecut) {
          m.push_back(a);
          m.push_back(b);
          m.push_back(d);
        }
      }
  return m;
}

}  // namespace

int main(int argc, char** argv) {
  if (argc < 2) {
    std::printf("FAIL 0 usage: host_check <input>\n");
    return 2;
  }
  std::ifstream in(argv[1]);
  double lat[9], A[2], C[2], alpha, ecut;
  int km[3], nsym;
  for (double& v : lat) in >> v;
  for (int& v : km) in >> v;
  in >> A[0] >> A[1] >> C[0] >> C[1] >> alpha >> ecut >> nsym;
  std::vector<int32_t> rot(size_t(9) * nsym);
  std::vector<double> tau(size_t(3) * nsym);
  for (int o = 0; o < nsym; ++o) {
    for (int i = 0; i < 9; ++i) in >> rot[9 * o + i];
    for (int i = 0; i < 3; ++i) in >> tau[3 * o + i];
  }
  int nq = 0, nkb = 0;
  in >> nq;
  std::vector<double> q2(nq);
  for (double& v : q2) in >> v;
  in >> nkb;
  std::vector<double> kb(size_t(3) * nkb);
  for (double& v : kb) in >> v;
  if (!in) {
    std::printf("FAIL 0 unreadable input\n");
    return 2;
  }

  tc_ctx ctx;   // device 0, no stream: only the calls that do no device work are made
  tc_ctx* c = &ctx;
  const double zero9[9] = {0};
  const double bad_a[2] = {-1.0, 1.0}, bad_c[2] = {1.0, 0.0};
  int32_t m_out[3] = {100, 0, 0};
  int32_t m_dup[6] = {0, 0, 0, 0, 0, 0};

  // calls before the problem is described, and bad arguments
  code("null_context", tc_set_cell(nullptr, lat));
  code("null_lattice", tc_set_cell(c, nullptr));
  code("degenerate_lattice", tc_set_cell(c, zero9));
  code("kmesh_zero", tc_set_kmesh(c, 0, 1, 1));
  code("kmesh_large", tc_set_kmesh(c, 17, 1, 1));
  code("grid_unsupported", tc_set_grid(c, 10, 10, 10));
  code("grid_not_cubic", tc_set_grid(c, 8, 8, 16));
  code("basis_before_mesh", tc_set_basis(c, 0, 1, m_dup));
  code("nspin_before_mesh", tc_set_nspin(c, 2));
  const double half[3] = {0.5, 0.5, 0.5}, one[3] = {1.0, 0.0, 0.0}, neg[3] = {-0.25, 0.0, 0.0};
  code("shift_before_mesh", tc_set_kmesh_shift(c, half));
  code("symmetry_before_mesh", tc_set_symmetry(c, 0, nullptr, nullptr));
  code("jastrow_null", tc_set_jastrow(c, nullptr, C));
  code("jastrow_negative_A", tc_set_jastrow(c, bad_a, C));
  code("jastrow_zero_C", tc_set_jastrow(c, A, bad_c));
  code("cusp_null", tc_set_jastrow_cusp(c, nullptr));
  code("cusp_negative_A", tc_set_jastrow_cusp(c, bad_a));
  code("options_precision", tc_set_options(c, 7, alpha, TC_DIV_PRINTED, ~0ull));
  code("options_alpha", tc_set_options(c, TC_PREC_FP64, 0.0, TC_DIV_PRINTED, ~0ull));
  code("options_div", tc_set_options(c, TC_PREC_FP64, alpha, 9, ~0ull));
  code("batch_negative", tc_set_batch(c, -1));
  EXPECT(std::strlen(tc_last_error(c)) > 0);

  // a complete description
  code("cell", tc_set_cell(c, lat));
  code("kmesh", tc_set_kmesh(c, km[0], km[1], km[2]));
  code("grid", tc_set_grid(c, 8, 8, 8));
  code("jastrow", tc_set_jastrow(c, A, C));
  code("options", tc_set_options(c, TC_PREC_FP64, alpha, TC_DIV_PRINTED, ~0ull));
  code("nspin_3", tc_set_nspin(c, 3));
  code("nspin_2", tc_set_nspin(c, 2));
  code("shift_null", tc_set_kmesh_shift(c, nullptr));
  code("shift_one", tc_set_kmesh_shift(c, one));
  code("shift_negative", tc_set_kmesh_shift(c, neg));
  code("shift", tc_set_kmesh_shift(c, half));
  {   // the shifted points and the unchanged mesh differences
    double f[3], g[3];
    ctx.pb.kfrac(ctx.pb.nk - 1, f);
    ctx.pb.kfrac_mesh(ctx.pb.nk - 1, g);
    for (int i = 0; i < 3; ++i) EXPECT(std::fabs(f[i] - g[i] - 0.5 / km[i]) < 1e-15);
  }
  const double sig_before = (gb_constant(ctx.pb), ctx.pb.sigma_aux);
  code("kmesh_again", tc_set_kmesh(c, km[0], km[1], km[2]));   // resets the shift
  EXPECT(ctx.pb.kshift[0] == 0.0 && ctx.pb.kshift[1] == 0.0 && ctx.pb.kshift[2] == 0.0);
  gb_constant(ctx.pb);
  EXPECT(ctx.pb.sigma_aux == sig_before);   // the Gygi-Baldereschi sum uses mesh differences only
  code("cusp", tc_set_jastrow_cusp(c, A));
  EXPECT(ctx.pb.C[0] == std::sqrt(2.0 * A[0]) && ctx.pb.C[1] == std::sqrt(A[1]));
  code("basis_index", tc_set_basis(c, ctx.pb.nk, 1, m_dup));
  code("basis_null", tc_set_basis(c, 0, 1, nullptr));
  code("basis_outside_grid", tc_set_basis(c, 0, 1, m_out));
  code("basis_duplicate", tc_set_basis(c, 0, 2, m_dup));
  int basis_ok = TC_OK;
  for (int k = 0; k < ctx.pb.nk; ++k) {
    const std::vector<int32_t> m = sphere(ctx.pb, k, ecut);
    const int st = tc_set_basis(c, k, int(m.size() / 3), m.data());
    if (st != TC_OK) basis_ok = st;
  }
  code("basis", basis_ok);
  EXPECT(ctx.pb.npw[0] > 0);

  // host tables: Gygi-Baldereschi constant and the Jastrow kernels with their exact tangents
  gb_constant(ctx.pb);
  std::printf("gb %.17g %.17g\n", ctx.pb.sigma_aux, ctx.pb.delta_gb);
  for (double Q2 : q2) {
    const Jk k = jastrow_ft(Q2, A[0], C[0]);
    std::printf("jk %.17g %.17g %.17g %.17g %.17g %.17g\n", Q2, A[0], C[0], k.u, k.lap, k.w);
  }
  for (int dir = 0; dir < 4; ++dir) {
    const double Q2 = q2.empty() ? 1.0 : q2[q2.size() / 2];
    const int ch = dir % 2;
    const double h = 1e-6;
    const TableVariant tp{TableVariant::TANGENT, dir, h}, tm{TableVariant::TANGENT, dir, -h};
    const Jk kp = chan_kernels(tp, A, C, ch, Q2), km2 = chan_kernels(tm, A, C, ch, Q2);
    double Ap[2] = {A[0], A[1]}, Am[2] = {A[0], A[1]}, Cp[2] = {C[0], C[1]}, Cm[2] = {C[0], C[1]};
    const double step = 1e-5 * (dir < 2 ? A[ch] : C[ch]);
    (dir < 2 ? Ap : Cp)[ch] += step;
    (dir < 2 ? Am : Cm)[ch] -= step;
    const Jk fp = jastrow_ft(Q2, Ap[ch], Cp[ch]), fm = jastrow_ft(Q2, Am[ch], Cm[ch]);
    std::printf("tangent %d %.17g %.17g\n", dir, (kp.u - km2.u) / (2 * h), (fp.u - fm.u) / (2 * step));
    std::printf("tangent %d %.17g %.17g\n", dir, (kp.w - km2.w) / (2 * h), (fp.w - fm.w) / (2 * step));
  }

  // symmetry: bad operations, then the given group and its k-point orbits
  if (nsym > 0) {
    std::vector<int32_t> r2(rot.begin(), rot.begin() + 9);
    r2[0] *= 2;   // det 2
    code("symmetry_det", tc_set_symmetry(c, 1, r2.data(), tau.data()));
    std::vector<double> t2(tau.begin(), tau.begin() + 3);
    t2[0] += 0.01;   // not a multiple of 1/N
    code("symmetry_tau", tc_set_symmetry(c, 1, rot.data(), t2.data()));
    code("symmetry_not_group", nsym > 2 ? tc_set_symmetry(c, 2, rot.data() + 9, tau.data() + 3) : TC_ERR_ARG);
    code("symmetry", tc_set_symmetry(c, nsym, rot.data(), tau.data()));
    std::vector<int> size(ctx.pb.nk, 0);
    for (int k = 0; k < ctx.pb.nk; ++k) {
      EXPECT(ctx.pb.krep[k] >= 0 && ctx.pb.krep[k] <= k);
      ++size[ctx.pb.krep[k]];
    }
    std::printf("sym %d", int(ctx.pb.irr.size()));
    for (int r : ctx.pb.irr) std::printf(" %d", size[r]);
    std::printf("\n");
    code("symmetry_off", tc_set_symmetry(c, 0, nullptr, nullptr));
  }

  // band k-points
  const double on_mesh[3] = {0.0, 0.0, 0.0};
  code("band_setter_takes_mesh_point", tc_set_band_kpoints(c, 1, on_mesh));   // rejected at application
  code("band_negative", tc_set_band_kpoints(c, -1, nullptr));
  if (nkb > 0) {
    code("band", tc_set_band_kpoints(c, nkb, kb.data()));
    code("band_basis_index", tc_set_band_basis(c, nkb, 1, m_dup));
  }
  // the triangular store of TC mode: row offsets (rows of min(t + 1, Q1) pairs) and the decode of pair p of
  // a target batch into its row and partner, against enumerating the rows
  {
    const int cases[][3] = {{8, 2, 3},     {12, 4, 6},     {12, 12, 12},  {256, 16, 256},
                            {256, 16, 208}, {256, 134, 256}, {1000, 37, 700}, {4096, 64, 4096}};
    long n = 0, bad = 0;
    for (const auto& cs : cases) {
      const int P = cs[0], T = cs[1], Q1 = cs[2];
      bad += tcmi::tri_row(P, P) != long(P) * (P + 1) / 2;
      for (int t0 = 0; t0 < P; t0 += T) {
        const int nt = std::min(T, P - t0);
        tcmi::MeshInfo mi{};
        mi.P = std::min(t0 + nt, Q1);
        mi.trq = Q1;
        long p = 0;
        for (int t = 0; t < nt; ++t)
          for (int q = 0; q < std::min(t0 + t + 1, Q1); ++q, ++p, ++n) {
            int tt = -1, qq = -1;
            tcmi::pair_tq(mi, t0, p, tt, qq);
            bad += tt != t || qq != q;
          }
        bad += p != tcmi::tri_row(t0 + nt, Q1) - tcmi::tri_row(t0, Q1);
      }
    }
    std::printf("tri %ld %ld\n", n, bad);
  }
  std::printf("done %d\n", g_fail);
  return g_fail == 0 ? 0 : 1;
}
