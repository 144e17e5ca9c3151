"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer (no device needed).

tests/native/host_check.cpp compiles the library's translation unit into a host program (sanitizers on
the host side only; the device code is reduced to the 8-point engine) and drives every entry point that
only describes the problem, with bad and good arguments, on the fcc cell with the diamond structure's
48 operations.  The test requires a clean sanitizer run, checks each status code against the header's
documented errors, and compares the host tables with the oracle and with closed facts:
  * the Gygi-Baldereschi sum and constant with the oracle's (Eq. correction2);
  * the Jastrow kernels u~, (lap u)~ and (grad u)^2~ with the oracle's closed forms (Sec. 2.6.3, App. B),
    including the small-g series branch;
  * the exact tangents of the kernels along A and C (dual numbers) with central differences;
  * the orbits of the 2x2x2 Gamma-centred mesh of the fcc lattice under O_h: Gamma, the four L-type
    and the three X-type points (3 representatives, orbit sizes 1, 3, 4);
  * the triangular pair store's row offsets and the z stage's decode of a pair into row and partner.
"""
import os
import subprocess

import numpy as np
import pytest
import torch

import tcinputs as T
from oracle.fftroute import Problem, jastrow_kernels

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "host_check.cpp")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

OK, ARG, STATE, GRID, KMESH, UNSUP = 0, -1, -2, -3, -4, -5
EXPECTED = {
    "null_context": ARG, "null_lattice": ARG, "degenerate_lattice": ARG, "kmesh_zero": KMESH,
    "kmesh_large": KMESH, "grid_unsupported": UNSUP, "grid_not_cubic": UNSUP, "basis_before_mesh": STATE,
    "nspin_before_mesh": STATE, "symmetry_before_mesh": STATE, "jastrow_null": ARG, "jastrow_negative_A": ARG,
    "jastrow_zero_C": ARG, "options_precision": ARG, "options_alpha": ARG, "options_div": ARG,
    "batch_negative": ARG, "cell": OK, "kmesh": OK, "grid": OK, "jastrow": OK, "options": OK, "nspin_3": ARG,
    "nspin_2": OK, "basis_index": ARG, "basis_null": ARG, "basis_outside_grid": GRID, "basis_duplicate": ARG,
    "basis": OK, "symmetry_det": ARG, "symmetry_tau": ARG, "symmetry_not_group": ARG, "symmetry": OK,
    "symmetry_off": OK, "band_setter_takes_mesh_point": OK, "band_negative": ARG, "band": OK,
    "band_basis_index": ARG, "shift_before_mesh": STATE, "cusp_null": ARG, "cusp_negative_A": ARG,
    "shift_null": ARG, "shift_one": ARG, "shift_negative": ARG, "shift": OK, "kmesh_again": OK, "cusp": OK,
}


@pytest.fixture(scope="module")
def run(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("hostcheck")
    exe = str(d / "host_check")
    # sanitizers on the host side only (each -fsanitize after -Xarch_host); device code as in the library
    cmd = [HIPCC, "-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-DTCMI_HOST_CHECK_BUILD",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", SRC, "-o", exe]
    b = subprocess.run(cmd, capture_output=True, text=True)
    assert b.returncode == 0, b.stderr[-3000:]
    syms = subprocess.run(["nm", exe], capture_output=True, text=True).stdout
    assert "__asan_init" in syms and "__ubsan_handle" in syms   # both sanitizers are built in
    w = T.fcc_si(kmesh=(2, 2, 2))
    ops = T.diamond_ops(w.lattice)
    ops.sort(key=lambda o: (not np.array_equal(o[0], np.eye(3, dtype=int)) or np.any(o[1] != 0)))
    q2 = [1e-9, 0.01, 0.5, 2.0, 10.0]
    kb = [(0.1, 0.2, 0.3), (0.25, 0.0, 0.0)]
    lines = [" ".join(f"{x:.17g}" for x in np.asarray(w.lattice, float).reshape(-1)),
             " ".join(str(x) for x in w.kmesh),
             f"{w.A[0]:.17g} {w.A[1]:.17g} {w.C[0]:.17g} {w.C[1]:.17g} {w.alpha:.17g} 1.2",
             str(len(ops))]
    for R, tau in ops:
        lines.append(" ".join(str(int(x)) for x in np.asarray(R).reshape(-1)) + " " +
                     " ".join(f"{x:.17g}" for x in tau))
    lines += [str(len(q2)), " ".join(f"{x:.17g}" for x in q2), str(len(kb))]
    lines += [" ".join(f"{x:.17g}" for x in k) for k in kb]
    inp = d / "input.txt"
    inp.write_text("\n".join(lines) + "\n")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe, str(inp)], capture_output=True, text=True, env=env, timeout=300)
    return w, q2, r


def test_clean_sanitizer_run(run):
    _, _, r = run
    assert "AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-3000:]
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-2000:])
    assert "FAIL" not in r.stdout
    assert r.stdout.strip().splitlines()[-1] == "done 0"


def test_status_codes_are_the_documented_ones(run):
    _, _, r = run
    got = {ln.split()[1]: int(ln.split()[2]) for ln in r.stdout.splitlines() if ln.startswith("code ")}
    assert got == EXPECTED


def test_gygi_baldereschi_constant_equals_the_oracle(run):
    w, _, r = run
    sig, dgb = [float(x) for x in next(ln for ln in r.stdout.splitlines() if ln.startswith("gb ")).split()[1:]]
    pr = Problem(w)
    assert sig == pytest.approx(pr.sigma_aux, rel=1e-12)
    assert dgb == pytest.approx(pr.delta_gb, rel=1e-12)


def test_jastrow_kernels_equal_the_oracle(run):
    _, q2, r = run
    rows = [[float(x) for x in ln.split()[1:]] for ln in r.stdout.splitlines() if ln.startswith("jk ")]
    assert len(rows) == len(q2)
    for Q2, A, C, u, lap, wk in rows:
        ut, lp, W = jastrow_kernels(torch.tensor([Q2], dtype=torch.float64), A, C)
        for a, b in ((u, ut), (lap, lp), (wk, W)):
            assert a == pytest.approx(float(b[0]), rel=1e-12, abs=1e-300)


def test_kernel_tangents_equal_central_differences(run):
    _, _, r = run
    rows = [[float(x) for x in ln.split()[2:]] for ln in r.stdout.splitlines() if ln.startswith("tangent ")]
    assert len(rows) == 8
    for exact, fd in rows:
        assert exact == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_triangular_pair_store_rows_and_decode(run):
    """The triangular store's rows and the z stage's decode of a batch's pair index into (row, partner)
    agree with enumerating the rows, for whole and partial stores and batches that do not divide P."""
    _, _, r = run
    n, bad = (int(x) for x in next(ln for ln in r.stdout.splitlines() if ln.startswith("tri ")).split()[1:])
    assert n > 8_000_000 and bad == 0


def test_fcc_mesh_orbits_under_the_diamond_group(run):
    _, _, r = run
    f = next(ln for ln in r.stdout.splitlines() if ln.startswith("sym ")).split()[1:]
    assert int(f[0]) == 3
    assert sorted(int(x) for x in f[1:]) == [1, 3, 4]
