"""Throughput of the electrode-charge step on one MI355X.

A step is one pass of the hot path over one batch of synthetic frames:
cpm_rhs (b = chi - b_sol for F electrolyte frames) followed by cpm_solve
(warm start, block CG, electroneutrality projection) for those F frames,
with E assembled once beforehand (its assembly is timed and reported
separately as GFLOP/s). Inputs are resident in HBM before the timed region.

Prints one JSON line (progress on stderr). Default workload 5: two 4-layer
AB-graphite electrodes, N = 131072 electrode atoms, 32 frames of 200000
random +-1 e ions, a = 1.979 /A, beta = 0.3 /A, rcut = 12 A, k-space
accuracy 1e-6 (482337 k-vectors), 1 V; E stored in FP64 (137 GB, the
residual and the FP64 reference), FP32 (69 GB, the inner solves of the
headline) and BF16 (34 GB, the BF16 variant reported as a mode).
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
# plain copy run after the timed region: its counter readings calibrate the
# FETCH_SIZE / WRITE_SIZE counters (bytes moved are known exactly)
CALIB_BYTES = 1 << 30
K_E = 14.3996454784   # V*A/e: cpm_rhs divides chi by it, so 1 V is 1/K_E in b units
# 16 columns run on the row-split kernel
KERNEL_OF_KIND = {"matvec_f64": "block_matvec_rows_kernel<double>",
                  "matvec_f32": "block_matvec_rows_kernel<float>",
                  "matvec_bf16": "block_matvec_rows_kernel<unsigned short>"}
# 32..64 columns of an FP32 / BF16 E run on the split-bf16 kernel
KERNEL_OF_KIND_WIDE = {"matvec_f64": "block_matvec_f64s_kernel<{ng}>",
                       "matvec_f32": "block_matvec_split_kernel<float, {ng}>",
                       "matvec_bf16": "block_matvec_split_kernel<unsigned short, {ng}>"}


# the ion structure factors of the right-hand side (|n_z| <= 47: every workload here)
SF_KERNEL = "sf_gemm_kernel"


def kernel_name(kind, ng):
    if kind == "sf":
        return SF_KERNEL
    return (KERNEL_OF_KIND_WIDE if ng >= 2 else KERNEL_OF_KIND)[kind].format(ng=ng)


CSRC = os.path.join(ROOT, "paper_2111_06704_amd", "csrc")


def kernel_source(name):
    """The source file that defines a kernel of the traffic record."""
    return os.path.join(CSRC, "rhs.hip" if name.startswith(SF_KERNEL) else "cg.hip")
PROFILE_STRIDE = 5   # timed launches of the block product: every 5th (coprime to the check batches)
MODE_STEPS = 5       # timed steps of every comparison mode (at most --steps)
# in-plane patch edge (A) of the coarse-space correction per workload (0: off).
# Sweeps of the FP32 solve to 1e-11 over edges 18 .. 5 A and checks every 8 / 4
# / 2 iterations: workload 5 704 ms (48 iterations, P alone) -> 255 ms at 9 A
# (4080 patches, 10 iterations, checks every 2); workload 3 74 -> 38 ms at 14 A
# (480 patches, 12 iterations, checks every 4); workload 2 (N = 4608) is
# faster without it (1.64 ms against 2.1 ms: the seven extra launches per
# iteration cost more than the 8 iterations they save)
COARSE_EDGE = {3: 14.0, 5: 9.0}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", type=int, default=5, choices=[1, 2, 3, 5])
    ap.add_argument("--tol", type=float, default=1e-11)
    ap.add_argument("--check-every", type=int, default=None,
                    help="iterations per device-side convergence check (all modes; default 8 at "
                         "workload 5, 4 elsewhere)")
    ap.add_argument("--inner-tol", type=float, default=None,
                    help="reliable-update factor of the FP32 / BF16 modes (default: "
                         "1e-4 for FP32 with PCG-DC at workload 2, 1e-3 otherwise)")
    ap.add_argument("--precision", default="f32", choices=["f64", "f32", "bf16"])
    ap.add_argument("--warm", default="mlp", choices=["zero", "chi", "mlp"])
    ap.add_argument("--precond", default="dc", choices=["jacobi", "dc"],
                    help="preconditioner of the timed solves")
    ap.add_argument("--dc-g", type=float, default=None,
                    help="PCG-DC screening g (1/A); default 0.08 with r_cut 12 / 14 / 14 A at "
                         "workloads 2 / 3 / 5 (sweeps there), else 0.15 with 7; the paper: "
                         "0.083 with 8")
    ap.add_argument("--dc-rcut", type=float, default=None, help="PCG-DC cutoff (A)")
    ap.add_argument("--coarse-edge", type=float, default=None,
                    help="in-plane patch edge (A) of the coarse-space correction of the sparse "
                         "preconditioner; 0 turns it off (default: per workload, from sweeps)")
    ap.add_argument("--weights", default=None,
                    help="warm-start network (default: the one for the workload's geometry)")
    ap.add_argument("--kmax-override", type=float, default=0.0,
                    help="K_max (1/A) instead of the 1e-6 accuracy rule (counter runs of the "
                         "block products only: the reported step is then not the workload's)")
    ap.add_argument("--mode-steps", type=int, default=MODE_STEPS,
                    help="timed steps of each comparison mode")
    ap.add_argument("--all-modes", action="store_true",
                    help="also time the BF16 and Jacobi-preconditioned mixed modes")
    ap.add_argument("--extras", action="store_true",
                    help="also time the matrix-inversion, capacitance-matrix (GCD) and "
                         "boundary-corrected paths (N <= 10000)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-frames", type=int, default=2)
    ap.add_argument("--cpu-atoms", type=int, default=64,
                    help="sampled atoms of the oracle's stationarity check (workloads 3 and 5)")
    ap.add_argument("--jitter", type=float, default=0.0,
                    help="displace every electrode atom by U(-a, a) A per component (genericity check)")
    ap.add_argument("--overlap", action=argparse.BooleanOptionalAction, default=False,
                    help="compute the right-hand side of the next step on a second stream "
                         "while the current step is solved (independent frames only: in MD "
                         "the next frame's ions depend on this step's charges)")
    ap.add_argument("--traffic-record", default=None,
                    help="JSON written by --summarize-pmc (default: profiles/traffic_workload<W>.json)")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"), default=None,
                    help="summarise two rocprofv3 --pmc runs of this script (FETCH_SIZE, then "
                         "WRITE_SIZE) into a traffic record and exit")
    ap.add_argument("--out", default=None, help="output path of --summarize-pmc")
    return ap.parse_args()


def _sha256(path):
    with open(path, "rb") as fh:
        return hashlib.sha256(fh.read()).hexdigest()


def _read_counters(d, counter):
    """Per kernel name: list of counter values (one per dispatch) from every
    counter_collection.csv under directory d."""
    out = {}
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {d}")
    for fn in files:
        with open(fn, newline="") as fh:
            for row in csv.DictReader(fh):
                if row.get("Counter_Name") != counter:
                    continue
                out.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]))
    return out


def summarize_pmc(fetch_dir, write_dir, out_path):
    """Traffic record: mean FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of
    every block-product kernel, and the factors that turn each counter into
    bytes, from the calibration copy (CALIB_BYTES read, CALIB_BYTES written)."""
    fetch = _read_counters(fetch_dir, "FETCH_SIZE")
    write = _read_counters(write_dir, "WRITE_SIZE")

    def calib(d):
        # the copy kernel: the elementwise kernel whose mean reading is largest
        cands = {k: v for k, v in d.items() if "elementwise" in k or "copy" in k.lower()}
        if not cands:
            raise SystemExit("calibration copy kernel not found in the counter run")
        k = max(cands, key=lambda x: np.mean(cands[x]))
        return k, float(np.median(cands[k]))

    kf, cf = calib(fetch)
    kw, cw = calib(write)
    # the counter run's own bench line (written beside its directory): the
    # structure factors' traffic depends on its k-set
    run_cfg = {}
    run_json = fetch_dir.rstrip("/") + ".json"
    if os.path.exists(run_json):
        with open(run_json) as fh:
            c = json.loads(fh.read().strip().splitlines()[-1])["config"]
        run_cfg = {"n_kvec": c.get("n_kvec"), "kmax_override": c.get("kmax_override")}
    rec = {"counter_unit": "KiB per dispatch",
           "calibration": {"kernel_fetch": kf, "kernel_write": kw, "bytes": CALIB_BYTES,
                           "fetch_kib": cf, "write_kib": cw,
                           "fetch_factor": CALIB_BYTES / (cf * 1024.0),
                           "write_factor": CALIB_BYTES / (cw * 1024.0)},
           "source_sha256": {os.path.basename(f): _sha256(os.path.join(CSRC, f))
                             for f in ("cg.hip", "rhs.hip")},
           "run_config": run_cfg, "kernels": {}}
    for name in sorted(set(fetch) | set(write)):
        m = re.search(r"(block_matvec(?:_split|_rows|_f64s)?_kernel)<([^>]*)>", name)
        if m:
            key = m.group(1) + "<" + m.group(2) + ">"
        elif re.search(r"\b" + SF_KERNEL + r"\b", name):
            key = SF_KERNEL
        else:
            continue
        # median over dispatches: launches that the device-side control
        # turned into no-ops move no data and are not typical
        rec["kernels"][key] = {"dispatches": len(fetch.get(name, [])),
                               "fetch_kib": float(np.median(fetch[name])) if name in fetch else None,
                               "write_kib": float(np.median(write[name])) if name in write else None}
    with open(out_path, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")
    print(json.dumps(rec))


def traffic_bytes(record_path, kind, ng, n_kvec=None):
    """HBM bytes per launch of a kernel from a committed traffic record; None
    if there is none, the source file of that kernel has changed since the
    counters were taken, or (structure factors) the counter run used another
    k-set than this one."""
    if not record_path or not os.path.exists(record_path):
        return None
    with open(record_path) as fh:
        rec = json.load(fh)
    name = kernel_name(kind, ng)
    if kind == "sf" and rec.get("run_config", {}).get("n_kvec") != n_kvec:
        return None
    src = kernel_source(name)
    if rec.get("source_sha256", {}).get(os.path.basename(src)) != _sha256(src):
        return None
    k = rec["kernels"].get(name)
    if not k or k.get("fetch_kib") is None or k.get("write_kib") is None:
        return None
    c = rec["calibration"]
    return 1024.0 * (k["fetch_kib"] * c["fetch_factor"] + k["write_kib"] * c["write_factor"])




def oracle_cores():
    try:
        from threadpoolctl import threadpool_info
        return max([int(i.get("num_threads", 1)) for i in threadpool_info()] + [1])
    except Exception:
        return os.cpu_count() or 1


def cpu_baseline_full(geo, ipos, iq, chi, nframes, q_gpu):
    """The FP64 oracle on the host: E and its Cholesky factor once, then per
    frame b and the two-step solve. Returns the baseline record and the
    charge error of the GPU result on the sampled frames."""
    from oracle import cpm as ocpm
    from oracle import ewald as ew
    from paper_2111_06704_amd import workloads as wl
    km = ew.kmax_from_eps(wl.EWALD_SPLIT, wl.KSPACE_EPS)
    t0 = time.perf_counter()
    E = ew.ewald_matrix(geo.pos, geo.box, wl.GAUSS_INV_WIDTH, wl.EWALD_SPLIT, wl.RCUT, km)
    fac = ocpm.cholesky(E)
    _, d, _ = ocpm.neutralising_vector(fac, geo.n)
    t1 = time.perf_counter()
    b, qs = ew.rhs(geo.pos, wl.GAUSS_INV_WIDTH, ipos[:nframes], iq[:nframes], chi, geo.box,
                   wl.EWALD_SPLIT, wl.RCUT, km)
    t2 = time.perf_counter()
    q = ocpm.two_step(fac, b, qs, d)
    t3 = time.perf_counter()
    r2, rm = ocpm.rel_errors(q_gpu[:nframes], q)
    rec = {"value": nframes / (t3 - t1), "unit": "solves/s", "cores": oracle_cores(),
           "kind": "oracle",
           "sample": f"{nframes} frames of the same workload: b (direct Ewald) + Cholesky solve + "
                     f"two-step projection per frame; E assembly and its factorisation once "
                     f"({t1 - t0:.1f} s, not in the rate)",
           "setup_s": t1 - t0}
    return rec, float(r2.max()), float(rm.max()), (t2 - t1) / nframes, (t3 - t2) / nframes


def cpu_baseline_large(geo, ipos, iq, chi, q_gpu, b_gpu, natoms, nframes_w2):
    """Workloads whose FP64 E does not fit a host factorisation (N = 32768:
    8.6 GB and 2.6e14 flop to assemble; N = 131072: 137 GB, 1.7e16 flop).

    Parity: the oracle evaluates, for frame 0 of the GPU result, (E q)_i
    matrix-free and b_i by direct Ewald at sampled atoms; the constrained
    minimum of Eq. 28 has E q - b uniform (Eq. 29), so the spread of
    (E q)_i - b_i measures the solve error.
    Rate: the oracle's per-frame work (b by direct Ewald, the Cholesky
    two-step solve) timed on workload 2 and scaled by its operation counts,
    (N + M) n_k for b and N^2 for the triangular solves: an extrapolation,
    labelled as such."""
    from oracle import ewald as ew
    from paper_2111_06704_amd import workloads as wl
    km = ew.kmax_from_eps(wl.EWALD_SPLIT, wl.KSPACE_EPS)
    rng = np.random.default_rng(2024)
    at = np.sort(rng.choice(geo.n, natoms, replace=False))
    log(f"cpu leg: oracle stationarity of frame 0 at {natoms} sampled atoms")
    t0 = time.perf_counter()
    u = ew.potentials_factored(geo.pos, wl.GAUSS_INV_WIDTH, q_gpu[0], geo.box, wl.EWALD_SPLIT,
                               wl.RCUT, km, at=at)
    bo, qso = ew.rhs_factored(geo.pos[at], wl.GAUSS_INV_WIDTH, ipos[0], iq[0], chi[at], geo.box,
                              wl.EWALD_SPLIT, wl.RCUT, km)
    t_check = time.perf_counter() - t0
    dev = u - bo
    spread = float(np.max(np.abs(dev - dev.mean())))
    bnorm = float(np.linalg.norm(b_gpu[0]))
    parity = {"frame": 0, "atoms": natoms, "stationarity_spread": spread,
              "stationarity_spread_over_b2": spread / bnorm,
              "b_relmax_sampled": float(np.max(np.abs(b_gpu[0, at] - bo)) / np.max(np.abs(bo))),
              "abs_sum_q_plus_qsol": float(abs(np.sum(q_gpu[0]) + qso)),
              "check_s": t_check}
    log(f"cpu leg: spread {spread:.3e} (|b|_2 {bnorm:.3e}) in {t_check:.1f} s; timing the oracle "
        f"on workload 2")
    geo2, ip2, iq2, chi2 = wl.workload(2, frames=nframes_w2)
    rec2, _, _, tb2, ts2 = cpu_baseline_full(geo2, ip2, iq2, chi2, nframes_w2,
                                             np.zeros((nframes_w2, geo2.n)))
    nk = len(ew.kvectors(geo.box, wl.EWALD_SPLIT, km)[0])
    nk2 = len(ew.kvectors(geo2.box, wl.EWALD_SPLIT, km)[0])
    m, m2 = ipos.shape[1], ip2.shape[1]
    fb = (geo.n + m) * nk / ((geo2.n + m2) * nk2)
    fs = (geo.n / geo2.n) ** 2
    t_frame = tb2 * fb + ts2 * fs
    rec = {"value": 1.0 / t_frame, "unit": "solves/s", "cores": rec2["cores"], "kind": "oracle",
           "extrapolated": True,
           "sample": f"oracle timed on {nframes_w2} frames of workload 2 (b by direct Ewald "
                     f"{tb2:.3f} s/frame, Cholesky two-step solve {ts2:.4f} s/frame, after "
                     f"{rec2['setup_s']:.1f} s of E assembly and factorisation) and scaled to this "
                     f"workload by (N + M) n_k (x{fb:.1f}) and N^2 (x{fs:.1f}); measured here: the "
                     f"oracle's matrix-free stationarity check of 1 frame at {natoms} atoms "
                     f"({t_check:.1f} s)",
           "setup_s": rec2["setup_s"]}
    return rec, parity


def main():
    t_start = time.perf_counter()
    args = parse()
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1],
                      args.out or os.path.join(ROOT, "profiles", f"traffic_workload{args.workload}.json"))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(json.dumps({"error": "the path runs on one GPU; --gpus must be 1"}))
        log("bench.py: only --gpus 1 is supported (the library runs on one GPU)")
        sys.exit(2)
    # one line per assembled k chunk on stderr (workload 5 assembles for minutes)
    os.environ.setdefault("CPM_PROGRESS", "1")
    import torch
    from paper_2111_06704_amd import cpm, warmstart, workloads as wl

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    cfg = args.workload
    if args.coarse_edge is None:
        args.coarse_edge = COARSE_EDGE.get(cfg, 0.0)
    # checks every 8 iterations suit workload 5 with P alone (48 iterations);
    # with the coarse space the residual falls about tenfold per iteration and
    # the recursive FP32 residual must be checked (and replaced) every 2
    ce_plain = 8 if cfg == 5 else 4
    if args.check_every is None:
        args.check_every = (2 if args.coarse_edge > 0 else 8) if cfg == 5 else 4
    # PCG-DC: the apply is cheap next to the product at large N, so a wide P
    # pays. Sweeps of (g, r_cut) over (0.15, 7) .. (0.06, 16) on each
    # workload (FP32 iterations to 1e-11): workload 5 80 at (0.15, 7), 64 at
    # (0.10, 10), 56 at 12 A, 48 at (0.08, 14) (solve 1132 -> 763 ms; 16 A no
    # better); workload 3 52 -> 32 at (0.08, 14) (84.9 -> 74.1 ms); workload 2
    # 32 -> 24 at (0.08, 12), 1.78 -> 1.74 ms (its apply is half the product's
    # time, so 14 A is slower there)
    if args.dc_g is None:
        args.dc_g = 0.08 if cfg in (2, 3, 5) else 0.15
    if args.dc_rcut is None:
        args.dc_rcut = {2: 12.0, 3: 14.0, 5: 14.0}.get(cfg, 7.0)
    geo, ipos, iq, chi = wl.workload(cfg)
    if args.jitter > 0:
        # genericity check: the same workload with every electrode atom displaced
        # by U(-jitter, jitter) per component (no lattice structure to exploit)
        geo = wl.jitter(geo, args.jitter, 7_000_000 + cfg)
    nf, m = ipos.shape[0], ipos.shape[1]
    log(f"workload {cfg}: N={geo.n} frames={nf} ions={m}")

    store = ("f32",)
    # workload 5 is quoted with the FP32 E and its BF16 variant: both stored
    if args.precision == "bf16" or cfg == 5 or (args.all_modes and cfg <= 3):
        store = ("f32", "bf16")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S = cpm.System(geo.pos, geo.box, wl.GAUSS_INV_WIDTH, wl.EWALD_SPLIT, wl.RCUT, wl.KSPACE_EPS,
                   kmax_override=args.kmax_override, store=store, profile_build=True)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t0
    prof_build = S.profile_read()[3]
    desc = S.describe()
    asm_gflops = prof_build["work"] / (prof_build["ms"] * 1e-3) / 1e9 if prof_build["ms"] > 0 else None
    log(f"E built in {build_s:.1f} s; contraction {prof_build['ms']:.1f} ms, "
        f"{asm_gflops:.1f} GFLOP/s; n_kvec={desc['n_kvec']}, device bytes {desc['device_bytes']}")

    t_ipos = torch.tensor(ipos, device=dev)
    t_iq = torch.tensor(iq, device=dev)
    t_chi = torch.tensor(chi, device=dev)
    b = torch.empty((nf, geo.n), dtype=torch.float64, device=dev)
    qsol = torch.empty((nf,), dtype=torch.float64, device=dev)
    q = torch.empty_like(b)

    prec = {"f64": cpm.PREC_F64, "f32": cpm.PREC_F32, "bf16": cpm.PREC_BF16}[args.precision]
    pcmode = cpm.PRECOND_DC if args.precond == "dc" else cpm.PRECOND_JACOBI
    # PCG-DC is built in every run: the FP64 reference with the same
    # preconditioner needs it, and d' is solved with it
    t0 = time.perf_counter()
    S.precond_dc(args.dc_g, args.dc_rcut)
    precond_build_s = time.perf_counter() - t0
    log(f"PCG-DC preconditioner built in {precond_build_s:.2f} s")
    coarse_m, coarse_build_s = 0, 0.0
    if args.coarse_edge > 0:
        t0 = time.perf_counter()
        coarse_m = S.precond_coarse(args.coarse_edge)
        torch.cuda.synchronize()
        coarse_build_s = time.perf_counter() - t0
        log(f"coarse space: {coarse_m} patches of edge {args.coarse_edge} A in {coarse_build_s:.2f} s")
    t0 = time.perf_counter()
    S.set_warm_chi(t_chi, preconditioner=cpm.PRECOND_DC)
    torch.cuda.synchronize()
    log(f"d' and the q_chi start in {time.perf_counter() - t0:.2f} s")
    weights = args.weights or warmstart.weights_for(cfg)
    warmstart.load_into(S, geo, weights)
    wmode = {"zero": cpm.WARM_ZERO, "chi": cpm.WARM_CHI, "mlp": cpm.WARM_MLP}[args.warm]

    def inner_tol_for(precision, pcm, override=None):
        # reliable-update factor: 1e-4 for FP32 with PCG-DC at workload 2
        # (from a sweep: one true residual fewer at the same 32 iterations),
        # 3e-3 at workload 5 (with P alone a sweep of 1e-1 .. 3e-3 and checks
        # every 4 / 8 gave the fewest true residuals at 3e-3 with 8; factors
        # of 1e-4 and below need more iterations, 1e-5 nearly three times as
        # many; with the coarse space 3e-3 and 1e-2 need the same 10-12
        # iterations and true residuals), 1e-3 elsewhere (BF16, Jacobi and
        # workload 3 need more iterations at 1e-4)
        if override is not None:
            return override
        if args.inner_tol is not None:
            return args.inner_tol
        if precision == cpm.PREC_F32 and pcm == cpm.PRECOND_DC and cfg == 2:
            return 1e-4
        return 3e-3 if cfg == 5 else 1e-3

    def solver(precision, wm, qout, pcm, inner=None, check_every=None):
        ce = check_every or args.check_every
        return lambda bb, qq: S.solve(bb, qq, tol=args.tol, precision=precision, warm_start=wm,
                                      inner_tol=inner_tol_for(precision, pcm, inner),
                                      check_every=ce, q_out=qout, preconditioner=pcm)

    # Steps: right-hand side of the batch, then its solve. With --overlap the
    # right-hand side of step k + 1 is computed on a second stream (default
    # priority) while step k is solved: the two share no memory in the
    # library, the b buffers alternate, and events order each buffer's reuse.
    main_stream = torch.cuda.current_stream()
    rhs_stream = torch.cuda.Stream()
    bufs = [(b, qsol), (torch.empty_like(b), torch.empty_like(qsol))]
    ev_rhs = [torch.cuda.Event(), torch.cuda.Event()]
    ev_used = [torch.cuda.Event(), torch.cuda.Event()]

    def enqueue_rhs(k):
        bb, qq = bufs[k % 2]
        with torch.cuda.stream(rhs_stream):
            rhs_stream.wait_event(ev_used[k % 2])
            S.set_stream()
            S.rhs(t_ipos, t_iq, t_chi, b_out=bb, qsol_out=qq)
            ev_rhs[k % 2].record(rhs_stream)
        S.set_stream()

    def run_steps(n, solve_fn, name=None):
        """n steps; returns the last solve's result."""
        last = None
        if not args.overlap:
            for k in range(n):
                S.rhs(t_ipos, t_iq, t_chi, b_out=b, qsol_out=qsol)
                last = solve_fn(b, qsol)
                if name and nf * geo.n > 1 << 22:
                    log(f"  {name}: step {k + 1}/{n}, {last[1]['iterations']} iterations")
            return last
        enqueue_rhs(0)
        for k in range(n):
            if k + 1 < n:
                enqueue_rhs(k + 1)
            main_stream.wait_event(ev_rhs[k % 2])
            last = solve_fn(*bufs[k % 2])
            ev_used[k % 2].record(main_stream)
        return last

    hname = f"{args.precision}_{args.precond}_{args.warm}"
    log(f"headline mode {hname}: {args.warmup} warm-up + {args.steps} timed steps")
    run_steps(max(1, args.warmup), solver(prec, wmode, q, pcmode), "warm-up")
    torch.cuda.synchronize()
    # every PROFILE_STRIDE-th launch of the block product is bracketed with HIP
    # events (the bracketing launch costs the host ~10 us more than a plain one)
    S.profile_enable(True, stride=PROFILE_STRIDE)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, st = run_steps(args.steps, solver(prec, wmode, q, pcmode), hname)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = S.profile_read()
    S.profile_enable(False)
    ms_per_step = elapsed / args.steps * 1e3
    value = nf * args.steps / elapsed
    log(f"headline: {value:.2f} solves/s, {st['iterations']} iterations")

    # the right-hand side alone (the same in every mode)
    nrhs = max(1, min(args.steps, args.mode_steps))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(nrhs):
        S.rhs(t_ipos, t_iq, t_chi, b_out=b, qsol_out=qsol)
    torch.cuda.synchronize()
    rhs_ms = (time.perf_counter() - t0) / nrhs * 1e3

    # comparison modes, each timed over the same number of steps
    nmode = max(1, min(args.steps, args.mode_steps))
    q64 = torch.empty_like(b)
    mode_list = [("f64_jacobi_zero", cpm.PREC_F64, cpm.WARM_ZERO, cpm.PRECOND_JACOBI, q64),
                 ("f64_dc_zero", cpm.PREC_F64, cpm.WARM_ZERO, cpm.PRECOND_DC, None),
                 ("f32_dc_zero", cpm.PREC_F32, cpm.WARM_ZERO, cpm.PRECOND_DC, None),
                 ("f32_dc_chi", cpm.PREC_F32, cpm.WARM_CHI, cpm.PRECOND_DC, None)]
    if args.all_modes:
        mode_list += [("f32_jacobi_zero", cpm.PREC_F32, cpm.WARM_ZERO, cpm.PRECOND_JACOBI, None),
                      ("f32_jacobi_mlp", cpm.PREC_F32, cpm.WARM_MLP, cpm.PRECOND_JACOBI, None),
                      ("f32_dc_mlp_again", cpm.PREC_F32, cpm.WARM_MLP, cpm.PRECOND_DC, None)]
        if "bf16" in store and cfg != 5:
            mode_list += [("bf16_dc_zero", cpm.PREC_BF16, cpm.WARM_ZERO, cpm.PRECOND_DC, None),
                          ("bf16_dc_mlp", cpm.PREC_BF16, cpm.WARM_MLP, cpm.PRECOND_DC, None)]
    # per-mode solver settings: the BF16 variant of workload 5 restarts its
    # inner CG on true residuals; a sweep (inner 1e-1 .. 1e-2, checks every
    # 4 / 8 iterations) gave the shortest solve at 1e-2 with checks every 4
    mode_opts = {"f64_jacobi_zero": dict(check_every=ce_plain)}
    if coarse_m:
        # the same mode as the headline with P alone (and its own check
        # interval): what the coarse space gains
        mode_list.append((f"{hname}_without_coarse", prec, wmode, pcmode, None))
        mode_opts[f"{hname}_without_coarse"] = dict(coarse=False, check_every=ce_plain)
    if cfg == 5 and "bf16" in store:
        mode_list.append(("bf16_dc_mlp", cpm.PREC_BF16, cpm.WARM_MLP, cpm.PRECOND_DC, None))
        mode_opts["bf16_dc_mlp"] = dict(inner=1e-2, check_every=4)
    modes = {}
    qm = torch.empty_like(b)
    for name, pm, wm, pcm, qout in mode_list:
        log(f"mode {name}: {nmode} timed steps")
        opts = dict(mode_opts.get(name, {}))
        coarse_off = not opts.pop("coarse", True)
        if coarse_off:
            S.precond_coarse(0.0)
        torch.cuda.synchronize()
        tm = time.perf_counter()
        _, sm = run_steps(nmode, solver(pm, wm, qout if qout is not None else qm, pcm, **opts),
                          name)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - tm) / nmode
        if coarse_off:
            S.precond_coarse(args.coarse_edge)
        modes[name] = {"solves_per_s": nf / dt, "ms_per_step": dt * 1e3,
                       "solve_only_solves_per_s": nf / (dt - rhs_ms * 1e-3),
                       "iterations": sm["iterations"], "true_residual_updates": sm["outer"],
                       "initial_rel_resid": sm["initial_rel_resid"], "steps": nmode,
                       "max_rel_resid": sm["max_rel_resid"]}
        if name in mode_opts:
            modes[name].update({k: v for k, v in mode_opts[name].items()})
        log(name, modes[name])
    fp64 = modes["f64_jacobi_zero"]
    fp64dc = modes["f64_dc_zero"]

    extras = {}
    if args.extras and geo.n <= 10000:
        extras = run_extras(S, cpm, wl, geo, args, b, qsol, q64, dev, t_ipos, t_iq, t_chi, nf,
                            prec, pcmode, inner_tol_for, run_steps)

    # rooflines from the live HIP-event timing of the timed region (every
    # PROFILE_STRIDE-th launch of each kind): the block matrix product with
    # the most time (HBM-bound: algorithmic bytes) and the ion structure
    # factors of the right-hand side (FP64 matrix cores: algorithmic flops);
    # `roofline` is whichever of the two takes more of the step
    kinds = {0: "matvec_f64", 1: "matvec_f32", 2: "matvec_bf16", 4: "sf"}
    ng = min(4, (nf + 15) // 16)
    rec_path = args.traffic_record or os.path.join(ROOT, "profiles", f"traffic_workload{cfg}.json")

    def roofline_of(k):
        launches = max(1, prof[k]["launches"])
        avg_ms = prof[k]["ms"] / launches
        work = prof[k]["work"] / launches
        r = {"traffic": traffic_bytes(rec_path, kinds[k], ng, desc["n_kvec"]),
             "traffic_unit": "bytes per launch",
             "kernel": kernel_name(kinds[k], ng), "avg_launch_us": avg_ms * 1e3,
             "launches": prof[k]["launches"], "timed_every": PROFILE_STRIDE,
             "kernel_share_of_step": PROFILE_STRIDE * prof[k]["ms"] / (elapsed * 1e3)}
        if k == 4:
            achieved = work / (avg_ms * 1e-3) / 1e12
            r.update({"bound": "mfma", "achieved": achieved, "peak": FP64_PEAK_TFLOPS,
                      "unit": "TFLOP/s", "frac": achieved / FP64_PEAK_TFLOPS,
                      "flops_per_launch": work})
        else:
            achieved = work / (avg_ms * 1e-3) / 1e9
            r.update({"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": achieved / HBM_PEAK_GBS, "bytes_per_launch": work})
        return {key: r[key] for key in ("bound", "achieved", "peak", "unit", "frac", "traffic")} | r

    kmv = max((0, 1, 2), key=lambda i: prof[i]["ms"])
    roofline_mv = roofline_of(kmv)
    roofline_sf = roofline_of(4) if prof[4]["launches"] else None
    roofline = roofline_sf if roofline_sf and prof[4]["ms"] > prof[kmv]["ms"] else roofline_mv

    # counter calibration: a plain copy of CALIB_BYTES (outside the timed region)
    src = torch.ones(CALIB_BYTES // 8, dtype=torch.float64, device=dev)
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)   # an elementwise kernel, never a DMA copy
    torch.cuda.synchronize()
    # the same copy timed: the bandwidth a plain streaming kernel reaches here
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(5):
        torch.mul(src, 1.0, out=dst)
    ev1.record()
    torch.cuda.synchronize()
    copy_gbs = 2.0 * CALIB_BYTES * 5 / (ev0.elapsed_time(ev1) * 1e-3) / 1e9
    roofline_mv["copy_kernel_GBps"] = copy_gbs
    roofline_mv["frac_of_copy"] = roofline_mv["achieved"] / copy_gbs
    del src, dst

    qg = q.cpu().numpy()
    q64g = q64.cpu().numpy()
    bg = b.cpu().numpy()
    rel_vs_fp64 = float(np.max(np.linalg.norm(qg - q64g, axis=1) / np.linalg.norm(q64g, axis=1)))
    out = {
        "metric": "charge solves/sec to 1e-8 rel (mixed+warm vs FP64 CG); E-assembly GFLOP/s",
        "value": value, "unit": "solves/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if prec == cpm.PREC_F64 else f"{args.precision}+f64",
        "data": "synthetic",
        "config": {"workload": f"workload {cfg}: two graphite electrodes, N={geo.n}, "
                               f"{nf} frames x {m} ions",
                   "n_electrode": geo.n, "frames_per_step": nf, "ions": m,
                   "n_kvec": desc["n_kvec"], "tol": args.tol, "check_every": args.check_every,
                   "inner_tol": inner_tol_for(prec, pcmode), "precision": args.precision,
                   "overlap_rhs": bool(args.overlap), "jitter_A": args.jitter,
                   "warm_start": args.warm, "warm_start_weights": os.path.basename(weights),
                   "preconditioner": args.precond, "dc_g": args.dc_g, "dc_rcut": args.dc_rcut,
                   "coarse_edge": args.coarse_edge or None, "coarse_patches": coarse_m,
                   "kmax_override": args.kmax_override or None,
                   "E_stored": ["f64"] + list(store), "device_bytes": desc["device_bytes"]},
        "fp64_cg_solves_per_s": fp64["solves_per_s"],
        "fp64_cg_iterations": fp64["iterations"],
        "speedup_vs_fp64_cg": value / fp64["solves_per_s"],
        "fp64_pcgdc_solves_per_s": fp64dc["solves_per_s"],
        "fp64_pcgdc_iterations": fp64dc["iterations"],
        "speedup_vs_fp64_pcgdc": value / fp64dc["solves_per_s"],
        "rhs_ms_per_step": rhs_ms,
        "solve_only_solves_per_s": nf / (ms_per_step * 1e-3 - rhs_ms * 1e-3),
        "iterations": st["iterations"], "true_residual_updates": st["outer"], "modes": modes,
        "initial_rel_resid": st["initial_rel_resid"], "max_rel_resid": st["max_rel_resid"],
        "max_abs_sum_q": st["max_abs_sum_q"],
        "charge_rel_err_vs_fp64_gpu": rel_vs_fp64,
        "e_assembly_gflops": asm_gflops, "e_assembly_ms": prof_build["ms"],
        "e_assembly_frac_fp64_peak": (asm_gflops / 1e3 / FP64_PEAK_TFLOPS) if asm_gflops else None,
        "e_build_s": build_s, "precond_build_s": precond_build_s,
        "coarse_build_s": coarse_build_s,
        "roofline": roofline,
        "roofline_block_product": roofline_mv,
        "roofline_structure_factors": roofline_sf,
    }
    out.update(extras)
    if not args.no_cpu_baseline:
        if geo.n <= 10000:
            rec, r2, rm, _, _ = cpu_baseline_full(geo, ipos, iq, chi, args.cpu_frames, qg)
            out["cpu_baseline"] = rec
            out["charge_rel2_vs_oracle"] = r2
            out["charge_relmax_vs_oracle"] = rm
        elif not args.kmax_override:
            rec, parity = cpu_baseline_large(geo, ipos, iq, chi, qg, bg, args.cpu_atoms,
                                             args.cpu_frames)
            out["cpu_baseline"] = rec
            out["oracle_stationarity"] = parity
    out["wall_s"] = time.perf_counter() - t_start
    print(json.dumps(out))


def run_extras(S, cpm, wl, geo, args, b, qsol, q64, dev, t_ipos, t_iq, t_chi, nf, prec, pcmode,
               inner_tol_for, run_steps):
    """Matrix inversion (Sec. III.B.1), the capacitance matrix with prescribed
    electrode totals (Supplementary Eq. S14-S24) and the boundary-corrected
    path (Eq. 39), each timed over --mode-steps steps (N <= 10000 only)."""
    import torch
    out = {}
    nst = max(3, args.mode_steps)
    q64n = q64.cpu().numpy()
    # matrix-inversion path, the paper's choice for N < 1e4: S = E^-1 (I - 1 d^T)
    # built once by the block solver, one product per step
    t0 = time.perf_counter()
    S.mi_build(tol=1e-13, preconditioner=pcmode)
    torch.cuda.synchronize()
    mi_build_s = time.perf_counter() - t0
    qmi = torch.empty_like(b)
    mi_fn = lambda bb, qq: S.mi_solve(bb, qq, q_out=qmi)
    run_steps(1, mi_fn)
    torch.cuda.synchronize()
    tm = time.perf_counter()
    run_steps(nst, mi_fn)
    torch.cuda.synchronize()
    mi_s = (time.perf_counter() - tm) / nst
    qm = qmi.cpu().numpy()
    out["matrix_inversion"] = {
        "solves_per_s": nf / mi_s, "ms_per_step": mi_s * 1e3, "build_s": mi_build_s,
        "charge_rel_err_vs_fp64_gpu": float(np.max(np.linalg.norm(qm - q64n, axis=1)
                                                   / np.linalg.norm(q64n, axis=1)))}
    log("mi", out["matrix_inversion"])
    # galvanostatic constraint: C_E from the electrode-indicator solves, then
    # per step the charges under prescribed electrode totals (here the totals
    # of the FP64 reference charges, so they must come back equal to them)
    labels = geo.electrode.astype(np.int32)
    t0 = time.perf_counter()
    cmat, cdet, cjoint, _ = S.gcd_build(labels, 2, tol=1e-12, precision=cpm.PREC_F64,
                                        preconditioner=pcmode)
    torch.cuda.synchronize()
    gcd_build_s = time.perf_counter() - t0
    qtot = torch.tensor(np.stack([q64n[:, labels == a].sum(axis=1) for a in range(2)], axis=1),
                        device=dev)
    qgcd = torch.empty_like(b)
    dmu = torch.empty_like(qtot)
    gcd_fn = lambda bb, qq: S.gcd_solve(bb, qtot, tol=args.tol, precision=prec,
                                        preconditioner=pcmode, check_every=args.check_every,
                                        inner_tol=inner_tol_for(prec, pcmode), q_out=qgcd,
                                        dmu_out=dmu)
    run_steps(1, gcd_fn)
    torch.cuda.synchronize()
    tm = time.perf_counter()
    _, _, gst = run_steps(nst, gcd_fn)
    torch.cuda.synchronize()
    gcd_s = (time.perf_counter() - tm) / nst
    qgn = qgcd.cpu().numpy()
    out["gcd"] = {"solves_per_s": nf / gcd_s, "ms_per_step": gcd_s * 1e3, "build_s": gcd_build_s,
                  "iterations": gst["iterations"], "max_abs_total_err": gst["max_abs_sum_q"],
                  "capacitance_matrix_e_per_V": (cmat / K_E).tolist(),
                  "joint_capacitance_e_per_V": cjoint / K_E,
                  "charge_rel_err_vs_fp64_gpu": float(np.max(np.linalg.norm(qgn - q64n, axis=1)
                                                             / np.linalg.norm(q64n, axis=1)))}
    log("gcd", out["gcd"])
    # boundary correction of Eq. 39 (slab geometry): its own E, FP32 + PCG-DC
    t0 = time.perf_counter()
    S2 = cpm.System(geo.pos, geo.box, wl.GAUSS_INV_WIDTH, wl.EWALD_SPLIT, wl.RCUT,
                    wl.KSPACE_EPS, store=("f32",), slab=True)
    S2.precond_dc(args.dc_g, args.dc_rcut)
    if args.coarse_edge > 0:
        S2.precond_coarse(args.coarse_edge)
    torch.cuda.synchronize()
    slab_build_s = time.perf_counter() - t0
    b2, qs2, q2 = torch.empty_like(b), torch.empty_like(qsol), torch.empty_like(b)

    def slab_step():
        S2.rhs(t_ipos, t_iq, t_chi, b_out=b2, qsol_out=qs2)
        return S2.solve(b2, qs2, tol=args.tol, precision=cpm.PREC_F32, warm_start=cpm.WARM_ZERO,
                        inner_tol=inner_tol_for(cpm.PREC_F32, cpm.PRECOND_DC),
                        check_every=args.check_every, q_out=q2, preconditioner=cpm.PRECOND_DC)

    slab_step()
    torch.cuda.synchronize()
    tm = time.perf_counter()
    for _ in range(nst):
        _, sst = slab_step()
    torch.cuda.synchronize()
    slab_s = (time.perf_counter() - tm) / nst
    out["slab_correction"] = {"solves_per_s": nf / slab_s, "ms_per_step": slab_s * 1e3,
                              "build_s": slab_build_s, "precision": "f32+f64",
                              "warm_start": "zero", "iterations": sst["iterations"],
                              "max_rel_resid": sst["max_rel_resid"],
                              "max_abs_sum_q": sst["max_abs_sum_q"]}
    log("slab", out["slab_correction"])
    S2.close()
    return out


if __name__ == "__main__":
    main()
