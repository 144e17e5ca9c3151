"""Benchmark of the transcorrelated-operator hot path on one MI355X.

A step is one full application of the two- and three-body TC operator (all
terms, SCF-mesh divergence corrections, energy) to every occupied orbital.  The
default workload is the largest single-GPU configuration: the 2x2x2 supercell of
the diamond-lattice silicon-like cell (16 atoms, fcc a = 10.26 bohr), 2x2x2
Gamma-centred k-mesh, 32 occupied bands, ~2400 plane waves per k, 48^3 FFT grid
(65,536 same-spin orbital pairs).  The 4x4x4-k-mesh cell on the 24^3 grid (also
65,536 pairs) is timed beside it.  The orbital coefficients are resident in HBM
before the timed region; each step runs G->r, the Hartree-type fields, the
occupied-occupied pass, passes A and B, r->G, the FP64 corrections and the
energy reductions.

Prints one JSON line (rank 0).  Metric: orbital-pair TC applications per
second = N_pairs / (seconds per step), and the TC energy's error against the
FP64 oracle on a sample of the same cell and grid.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "orbital-pair TC applications/sec + TC energy error vs FP64 oracle (FP32 vs FP64)"
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of a kernel, from two rocprofv3 counter passes (FETCH_SIZE, then WRITE_SIZE) over
# one bench step, each scaled by what the counter reads for a plain 1 GiB device copy (FETCH x2, WRITE x1),
# averaged over the launches of the step.  Keyed by workload, kernel and the hash of the library sources
# the counters were taken on: any later change to those sources makes the figure stale (reported as null).
MEASURED_TRAFFIC = {
    ("fcc_si_x2_k222_g48", "k_fused_A<float,48>", "b6bcb0ba83dba4aa"): 3.4390e10,
}


def source_hash() -> str:
    """sha256 (16 hex) of the library's device/host sources and its C header, in file-name order."""
    import hashlib

    h = hashlib.sha256()
    d = os.path.join(HERE, "paper_2302_07420_amd", "csrc")
    for f in sorted(os.listdir(d)):
        if f.endswith((".hip", ".hpp", ".h")):
            with open(os.path.join(d, f), "rb") as fh:
                h.update(fh.read())
    with open(os.path.join(HERE, "include", "tcmi.h"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def describe(w) -> str:
    """The cell of a named workload in words."""
    if w.name.startswith("fcc_si_x2"):
        return "2x2x2 supercell (16 atoms) of the fcc a=10.26 bohr silicon-like cell"
    if w.name.startswith("fcc_si"):
        return "fcc a=10.26 bohr silicon-like cell (2 atoms)"
    return f"simple-cubic electron gas, {w.nelec_cell} electrons"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_op(w, precision, stream, symmetry=None):
    import torch
    import paper_2302_07420_amd as tc

    op = tc.TCOperator(0, stream)
    op.set_cell(w.lattice)
    op.set_kmesh(*w.kmesh)
    op.set_grid(*w.grid)
    for ik, m in enumerate(w.miller):
        op.set_basis(ik, m)
    op.set_jastrow(w.A, w.C)
    op.set_options(precision, w.alpha, True, tc.TERM_ALL)
    if symmetry:
        op.set_symmetry(symmetry)
    # coefficients resident in HBM (torch owns the memory)
    keep = []
    for ik, c in enumerate(w.right):
        t = torch.from_numpy(c).to("cuda")
        keep.append(t)
        op.load_orbitals_dev(ik, t.data_ptr(), c.shape[0], w.occ[ik])
    torch.cuda.synchronize()
    return op, keep


def make_op_bitc(w, precision, stream):
    """Same problem shape in the biorthogonal mode (left orbitals loaded from the host; the library
    biorthogonalises them on the device before the timed region)."""
    import paper_2302_07420_amd as tc

    op = tc.TCOperator(0, stream)
    op.set_cell(w.lattice)
    op.set_kmesh(*w.kmesh)
    op.set_grid(*w.grid)
    for ik, m in enumerate(w.miller):
        op.set_basis(ik, m)
    op.set_jastrow(w.A, w.C)
    op.set_options(precision, w.alpha, True, tc.TERM_ALL)
    for ik in range(w.nk):
        op.load_orbitals(ik, w.right[ik], w.occ[ik], left=w.left[ik])
    return op


def time_steps(op, out, steps, warmup, profile=False):
    import torch

    for _ in range(warmup):
        op.apply_dev(out.data_ptr())
        op.energy()
    torch.cuda.synchronize()
    if profile:
        op.kernel_stats(reset=True)
        op.set_profiling(True)
    stream = torch.cuda.current_stream()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall = time.perf_counter()
    t0.record(stream)
    energies = []
    for _ in range(steps):
        op.apply_dev(out.data_ptr())
        energies.append(op.energy())
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall
    ms = t0.elapsed_time(t1) / steps
    stats = op.kernel_stats(reset=True) if profile else None
    if profile:
        op.set_profiling(False)
    return ms, wall / steps * 1e3, energies, stats


def oracle_sample(workload: str):
    """A bounded sample of the workload that the FP64 oracle finishes in 10-30 s: the same cell, grid,
    Jastrow and basis cut, fewer orbital pairs."""
    import tcinputs as T

    if workload == "fcc_si_x2_k222_g48":
        # the 16-atom supercell on the 48^3 grid at Gamma only, 16 of its bands (256 pairs)
        w = T.fcc_si(kmesh=(1, 1, 1), grid=48, nb=16, supercell=2, seed_offset=4)
        return w, "2x2x2 supercell (16 atoms), 48^3 grid, ~2400 plane waves, Gamma only, 16 bands"
    # the cell on the 24^3 grid with a 2x2x2 k-mesh (1,024 pairs)
    return T.fcc_si(kmesh=(2, 2, 2)), "fcc a=10.26 bohr cell, 24^3 grid, 4 bands, 2x2x2 k-mesh"


def cpu_baseline(workload: str):
    """The FP64 oracle as it stands, timed on a bounded sample of the workload (oracle_sample)."""
    import torch
    from oracle.fftroute import Problem

    cores = len(os.sched_getaffinity(0))
    torch.set_num_threads(cores)
    w, what = oracle_sample(workload)
    t = time.perf_counter()
    with torch.no_grad():
        pr = Problem(w)
        E = float(pr.energy())
    dt = time.perf_counter() - t
    npairs = w.npairs
    return {
        "value": npairs / dt,
        "unit": "orbital-pair TC applications/s",
        "cores": torch.get_num_threads(),
        "kind": "oracle",
        "sample": f"{what} ({npairs} same-spin pairs, all terms, both spins, energy {E:.10f} Ha); {dt:.1f} s",
        "seconds": dt,
        "energy_Ha": E,
        "_workload": w,
    }


def energy_errors_vs_oracle(w, E_oracle, stream):
    """The TC energy of the oracle's sample from the GPU path in each precision, and its relative error
    against the oracle's FP64 energy of the same inputs."""
    import paper_2302_07420_amd as tc

    out = {"workload": w.name, "oracle_energy_Ha": E_oracle}
    for name, prec in (("fp32", tc.TC_PREC_FP32), ("fp32_splitbf16", tc.TC_PREC_FP32_SPLITBF16),
                       ("fp64", tc.TC_PREC_FP64)):
        op, keep = make_op(w, prec, stream)
        E = op.energy()[0]
        op.close()
        del keep
        out[name] = {"energy_Ha": E, "rel_err": abs(E - E_oracle) / abs(E_oracle)}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 GPU path")
    ap.add_argument("--no-split", action="store_true", help="skip the FP32 + split-BF16 (MFMA z-DFT) path")
    ap.add_argument("--no-bitc", action="store_true", help="skip the biorthogonal-mode side measurement")
    ap.add_argument("--no-scf", action="store_true", help="skip the block-Davidson SCF side measurement")
    ap.add_argument("--no-sym", action="store_true", help="skip the crystal-symmetry side measurement")
    ap.add_argument("--no-band", action="store_true", help="skip the band k-point side measurement")
    ap.add_argument("--workload", default="fcc_si_x2_k222_g48",
                    help="named workload: fcc_si_x2_k222_g48 (default), fcc_si_k444_g24, heg14_g16, heg54_twist2_g32")
    ap.add_argument("--no-g24", action="store_true", help="skip the 24^3 cell timed beside the headline")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="run one plain device copy of this many MiB first (calibrates HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the library has no multi-GPU path (asked for --gpus {args.gpus})",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import tcinputs as T
    import paper_2302_07420_amd as tc

    w = T.workload(args.workload)
    log(f"workload {w.name}: nk={w.nk} nb={w.nband} grid={w.grid} pairs={w.npairs}")
    side = torch.cuda.Stream()          # default priority; the library enqueues on this stream
    torch.cuda.set_stream(side)
    stream = side.cuda_stream
    out = torch.empty((w.nk, w.nband, max(m.shape[0] for m in w.miller)), dtype=torch.complex128, device="cuda")
    if args.copy_calib_mib > 0:
        n = args.copy_calib_mib << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copy calibration: {n} bytes read + {n} bytes written")
        del src, dst

    op32, keep32 = make_op(w, tc.TC_PREC_FP32, stream)
    ms32, wall32, e32, stats = time_steps(op32, out, args.steps, args.warmup, profile=True)
    E32 = e32[-1][0]
    tot, stages = op32.timing()
    log(f"fp32: {ms32:.2f} ms/step (wall {wall32:.2f}), E = {E32:.12f}")
    op32.close()   # its resident store holds most of the device
    del keep32

    split = None
    if not args.no_split:
        op_s, keep_s = make_op(w, tc.TC_PREC_FP32_SPLITBF16, stream)
        ms_s, wall_s, e_s, stats_s = time_steps(op_s, out, args.steps, args.warmup, profile=True)
        split = {"value": w.npairs / (ms_s / 1e3), "ms_per_step": ms_s, "energy_Ha": e_s[-1][0],
                 "kernels_ms_per_step": {k: v["ms"] / args.steps for k, v in stats_s.items() if v["ms"] > 0}}
        log(f"fp32+split-bf16: {ms_s:.2f} ms/step, E = {e_s[-1][0]:.12f}")
        op_s.close()
        del keep_s

    fp64 = None
    if not args.no_fp64:
        op64, keep64 = make_op(w, tc.TC_PREC_FP64, stream)
        ms64, wall64, e64, _ = time_steps(op64, out, 1 if w.grid[0] >= 48 else max(1, min(args.steps, 2)), 1)
        E64 = e64[-1][0]
        fp64 = {"value": w.npairs / (ms64 / 1e3), "ms_per_step": ms64, "energy_Ha": E64}
        log(f"fp64: {ms64:.2f} ms/step, E = {E64:.12f}")
        op64.close()
        del keep64

    g24 = None
    if not args.no_g24 and args.workload != "fcc_si_k444_g24":
        # the 4x4x4-k-mesh cell on the 24^3 grid (65,536 pairs), FP32, the headline's step and warm-up counts
        w24 = T.workload("fcc_si_k444_g24")
        out24 = torch.empty((w24.nk, w24.nband, max(m.shape[0] for m in w24.miller)), dtype=torch.complex128,
                            device="cuda")
        op24, keep24 = make_op(w24, tc.TC_PREC_FP32, stream)
        ms24, _, e24, st24 = time_steps(op24, out24, args.steps, args.warmup, profile=True)
        dom24 = max(st24.items(), key=lambda kv: kv[1]["ms"])
        g24 = {"workload": w24.name, "value": w24.npairs / (ms24 / 1e3), "ms_per_step": ms24, "energy_Ha": e24[-1][0],
               "dominant_kernel": dom24[0].replace("<R,N", "<float,24"),
               "dominant_kernel_GBps": dom24[1]["bytes"] / (dom24[1]["ms"] * 1e-3) / 1e9,
               "kernels_ms_per_step": {k: v["ms"] / args.steps for k, v in st24.items() if v["ms"] > 0}}
        log(f"fcc_si_k444_g24 fp32: {ms24:.2f} ms/step, E = {e24[-1][0]:.12f}")
        op24.close()
        del keep24, out24

    bitc = None
    if not args.no_bitc:
        wb = T.workload("fcc_si_k444_g24_bitc")
        out = torch.empty((wb.nk, wb.nband, max(m.shape[0] for m in wb.miller)), dtype=torch.complex128, device="cuda")
        res_b = {}
        for name, prec, nst in (("fp32", tc.TC_PREC_FP32, args.steps), ("fp64", tc.TC_PREC_FP64, 1)):
            op_b = make_op_bitc(wb, prec, stream)
            ms_b, _, e_b, st_b = time_steps(op_b, out, nst, 1, profile=name == "fp32")
            res_b[name] = (ms_b, e_b[-1][0], st_b)
            op_b.close()
        ms_b, e_b, st_b = res_b["fp32"]
        bitc = {"workload": wb.name, "value": wb.npairs / (ms_b / 1e3), "ms_per_step": ms_b, "energy_Ha": e_b,
                "fp64_ms_per_step": res_b["fp64"][0], "fp64_energy_Ha": res_b["fp64"][1],
                "energy_rel_err_fp32_vs_fp64": abs(e_b - res_b["fp64"][1]) / abs(res_b["fp64"][1]),
                "kernels_ms_per_step": {k: v["ms"] / args.steps for k, v in st_b.items() if v["ms"] > 0}}
        log(f"bitc fp32: {ms_b:.2f} ms/step, E = {e_b:.12f}; fp64 {res_b['fp64'][0]:.2f} ms/step")

    scf = None
    if not args.no_scf:
        # three block-Davidson iterations (pmax = 2: three applications to 256 trial vectors each, the
        # subspace diagonalisation, and the energy of the new orbitals) from the workload's orbitals
        op_c, keep_c = make_op(T.workload("fcc_si_k444_g24"), tc.TC_PREC_FP32, stream)
        op_c.energy()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        hist, nit = op_c.scf(max_iter=3, pmax=2, etol=1e-300, otol=0.0)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        scf = {"iterations": nit, "pmax": 2, "ms_per_iteration": dt / nit * 1e3,
               "energies_Ha": [float(x) for x in hist], "precision": "fp32"}
        log(f"scf: {dt / nit * 1e3:.1f} ms per block-Davidson iteration, energies {list(hist)}")
        op_c.close()
        del keep_c

    sym = None
    if not args.no_sym:
        # the same cell with orbitals invariant under the diamond structure's 48 operations: the
        # symmetry-reduced path (occupied-occupied rows and targets at the 8 representative k-points of
        # 64) against the unreduced path on the same inputs
        ws = T.workload("fcc_si_k444_g24_sym")
        out = torch.empty((ws.nk, ws.nband, max(m.shape[0] for m in ws.miller)), dtype=torch.complex128, device="cuda")
        ops = T.diamond_ops(ws.lattice)
        res_y = {}
        for name, prec, sops, nst in (("sym_fp32", tc.TC_PREC_FP32, ops, args.steps),
                                      ("full_fp32", tc.TC_PREC_FP32, None, args.steps),
                                      ("full_fp64", tc.TC_PREC_FP64, None, 1)):
            op_y, keep_y = make_op(ws, prec, stream, sops)
            ms_y, _, e_y, _ = time_steps(op_y, out, nst, 1)
            res_y[name] = (ms_y, e_y[-1][0])
            op_y.close()
            del keep_y
        ms_y, e_y = res_y["sym_fp32"]
        sym = {"workload": ws.name, "operations": len(ops), "representative_kpoints": 8,
               "value": ws.npairs / (ms_y / 1e3), "ms_per_step": ms_y, "energy_Ha": e_y,
               "unreduced_fp32_ms_per_step": res_y["full_fp32"][0],
               "speedup_vs_unreduced_fp32": res_y["full_fp32"][0] / ms_y,
               "energy_rel_err_vs_unreduced_fp64": abs(e_y - res_y["full_fp64"][1]) / abs(res_y["full_fp64"][1])}
        log(f"symmetry fp32: {ms_y:.2f} ms/step vs unreduced {res_y['full_fp32'][0]:.2f} ms/step, E = {e_y:.12f}")

    band = None
    if not args.no_band:
        # band structure: the operator of the mesh orbitals applied to 4 orbitals at each of 16 k-points on
        # L - Gamma - X (off the mesh), with the band forms of the divergence corrections; one application
        # includes the mesh densities and occupied-occupied pass
        import numpy as np

        wb = T.workload("fcc_si_k444_g24_band16")
        res_b = {}
        for name, prec, nst in (("fp32", tc.TC_PREC_FP32, max(1, min(args.steps, 3))), ("fp64", tc.TC_PREC_FP64, 1)):
            op_b, keep_b = make_op(wb, prec, stream)
            op_b.set_band(wb.band_k, wb.band_miller, wb.band_right, wb.band_occ)
            op_b.apply_band()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(nst):
                _, eps_b = op_b.apply_band()
            torch.cuda.synchronize()
            res_b[name] = ((time.perf_counter() - t0) / nst * 1e3, eps_b)
            op_b.close()
            del keep_b
        nbp = len(wb.band_k) * wb.band_right[0].shape[0] * wb.nk * wb.nband
        e32, e64 = res_b["fp32"][1], res_b["fp64"][1]
        band = {"workload": wb.name, "band_kpoints": len(wb.band_k), "orbitals_per_kpoint": wb.band_right[0].shape[0],
                "ms_per_application": res_b["fp32"][0], "fp64_ms_per_application": res_b["fp64"][0],
                "band_pairs_per_s": nbp / (res_b["fp32"][0] / 1e3),
                "band_energy_max_abs_err_fp32_vs_fp64_Ha": float(np.max(np.abs(e32 - e64))),
                "band_energies_fp64_Ha": [[float(x.real) for x in row] for row in e64]}
        log(f"band: {res_b['fp32'][0]:.1f} ms per application (fp64 {res_b['fp64'][0]:.1f}), "
            f"max |eps32 - eps64| = {band['band_energy_max_abs_err_fp32_vs_fp64_Ha']:.2e} Ha")

    # dominant kernel and its roofline (algorithmic bytes / event-timed duration)
    dom = max(stats.items(), key=lambda kv: kv[1]["ms"])
    name, st = dom
    avg_ms = st["ms"] / max(1, st["launches"])
    avg_bytes = st["bytes"] / max(1, st["launches"])
    achieved = avg_bytes / (avg_ms * 1e-3) / 1e9
    total_kernel_ms = sum(v["ms"] for v in stats.values()) / args.steps
    kname = name.replace("<R,N", "<float,%d" % w.grid[0])
    shash = source_hash()
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
            "traffic": MEASURED_TRAFFIC.get((args.workload, kname, shash)), "kernel": kname,
            "avg_launch_ms": avg_ms, "algorithmic_bytes_per_launch": avg_bytes,
            "launches_per_step": st["launches"] / args.steps, "source_hash": shash}
    per_kernel = {k: {"ms_per_step": v["ms"] / args.steps,
                      "GBps": (v["bytes"] / (v["ms"] * 1e-3) / 1e9) if v["ms"] > 0 and v["bytes"] > 0 else None}
                  for k, v in stats.items() if v["ms"] > 0}

    cpu = None
    if not args.no_cpu:
        try:
            cpu = cpu_baseline(args.workload)
            log(f"cpu oracle: {cpu['value']:.3f} pairs/s on {cpu['cores']} threads ({cpu['seconds']:.1f} s)")
        except Exception as e:  # the baseline is reported, never required
            log(f"cpu baseline failed: {e!r}")
    vs_oracle = None
    if cpu is not None:
        wo = cpu.pop("_workload")
        vs_oracle = energy_errors_vs_oracle(wo, cpu["energy_Ha"], stream)
        log("energy vs oracle on its sample: " + ", ".join(
            f"{k} {v['rel_err']:.2e}" for k, v in vs_oracle.items() if isinstance(v, dict)))

    res = {
        "metric": METRIC,
        "value": w.npairs / (ms32 / 1e3),
        "unit": "orbital-pair TC applications/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms32,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"{w.name}: {describe(w)}, {w.kmesh[0]}x{w.kmesh[1]}x{w.kmesh[2]} "
                        f"Gamma-centred k-mesh, {w.nband} occupied bands, "
                        f"{sum(m.shape[0] for m in w.miller) / w.nk:.1f} plane waves/k, {w.grid[0]}^3 grid, "
                        f"all two- and three-body TC terms + SCF-mesh GB corrections + energy",
            "n_pairs": w.npairs,
            "precision": "fp32 FFTs / pair products / kernel multiplies; fp64 partner sums, corrections, energies",
        },
        "energy_Ha": E32,
        "energy_rel_err_fp32_vs_fp64": (abs(E32 - fp64["energy_Ha"]) / abs(fp64["energy_Ha"])) if fp64 else None,
        "energy_rel_err_vs_oracle": vs_oracle["fp32"]["rel_err"] if vs_oracle else None,
        "energy_vs_oracle": vs_oracle,
        "fp64_gpu": fp64,
        "speedup_fp32_vs_fp64_gpu": (w.npairs / (ms32 / 1e3)) / fp64["value"] if fp64 else None,
        "fp32_splitbf16_gpu": dict(split, energy_rel_err_vs_fp64=(abs(split["energy_Ha"] - fp64["energy_Ha"])
                                                                  / abs(fp64["energy_Ha"])) if fp64 else None)
        if split else None,
        "fcc_si_k444_g24_fp32_gpu": g24,
        "bitc_fp32_gpu": bitc,
        "scf_davidson_gpu": scf,
        "symmetry_fp32_gpu": sym,
        "band_fp32_gpu": band,
        "stages_ms": dict(zip(tc.STAGES, stages)),
        "kernels_ms_per_step": per_kernel,
        "kernel_ms_per_step_total": total_kernel_ms,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
