"""Benchmark: velocity-node updates per second of the IMEX-SSP3(4,3,3) MP-9
lattice Boltzmann step on one MI355X, FP64 and FP32 storage.

Workload: 2D four-quadrant Riemann problem on 4096 x 4096 cells over [0,1]^2,
8 x 8 Gauss-Hermite velocities per distribution (phi and chi: 128 planes per
cell), K = 2 (gamma = 7/5), tau = 1e-7, dt = 0.5 dx / max|p| (CFL 0.5),
outflow walls; seeded quadrant states (synthetic, see workloads.py).

One step = the three fused stage passes over all 2^31 populations.  The
JSON line reports the FP64 throughput as ``value`` (the plain FP64 method),
the FP32-storage run beside it, per-pass HIP-event timings, the roofline of
the dominant pass, and the FP64 CPU oracle timed on a bounded patch.
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
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PMAX8 = 4.144547186125894  # largest root of He_8
HBM_PEAK_GBS = 8000.0      # MI355X HBM3E spec peak
XGMI_LINK_GBS = 153.0      # one MI355X xGMI link, spec figure (slab workload estimate only)
METRIC = "velocity-node updates/s per IMEX step, FP32 vs FP64, % of HBM roofline"
# Kernel sources whose hash ties a committed counter summary to the code it measured.
KERNEL_SOURCES = ("paper_1909_08390_amd/csrc/kernels.hip", "paper_1909_08390_amd/csrc/common.hpp",
                  "paper_1909_08390_amd/csrc/device.hpp")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "stage_passes_riemann4096_hbm_traffic.txt")
INSTS_FILE = os.path.join(ROOT, "profiles", "stage_passes_riemann4096_inst_mix.txt")
# VALU lane-instruction peak of MI355X: 256 CUs x 4 SIMDs x 16 lanes per cycle x 2.4 GHz.  An FP64 FMA and an
# unpacked FP32 FMA each take one lane-slot; the 157.3 TFLOP/s FP32 figure counts packed FP32 (two FMAs per slot),
# which this code does not use.
VALU_PEAK_T = 256 * 4 * 16 * 2.4e9 / 1e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pass_bytes(planes, cells, elem, nf):
    """Algorithmic HBM bytes of the three passes (plane-sets read/written,
    FP64 moment sets read/written); see the design notes."""
    ps = planes * cells * elem
    ms = nf * cells * 8
    return {"stage3": 2 * ps + 2 * ms, "stage4": 4 * ps + 3 * ms, "stage5": 3 * ps + 2 * ms}


def _strip_comments(text):
    """C++ source without comments, trailing blanks and blank lines: what
    the compiler sees (the sources hold no comment markers inside strings)."""
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    return "\n".join(line.rstrip() for line in text.splitlines() if line.strip())


def kernel_source_hash():
    """Hash of the kernel sources' code (comments left out), which ties a
    committed counter summary to the code it measured."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel)) as f:
            h.update(_strip_comments(f.read()).encode())
    return h.hexdigest()[:16]


def read_traffic(size):
    """HBM bytes per launch of each stage pass from the committed counter
    summary, keyed "f64 stage4" etc.; empty when the summary is missing, was
    taken at another size or on other kernel sources."""
    out = {}
    if not os.path.exists(TRAFFIC_FILE):
        return out
    meta = {}
    with open(TRAFFIC_FILE) as f:
        for line in f:
            line = line.strip()
            if line.startswith("source_sha256:"):
                meta["sha"] = line.split(":", 1)[1].strip()
            elif line.startswith("size:"):
                meta["size"] = int(line.split(":", 1)[1])
            elif line.startswith("pass "):
                # pass <prec> <stage>: fetch_kib=.. write_kib=.. traffic_bytes=..
                head, tail = line.split(":", 1)
                _, prec, stage = head.split()
                kv = dict(t.split("=") for t in tail.split())
                out[f"{prec} {stage}"] = float(kv["traffic_bytes"])
    if meta.get("sha") != kernel_source_hash() or meta.get("size") != size:
        return {}
    return out


def read_valu_per_vn(size):
    """VALU lane-instructions per velocity node of each stage pass ("f64
    stage4" etc.) from the committed instruction-mix summary; empty when it
    is missing, was taken at another size or on other kernel sources."""
    out, meta = {}, {}
    if not os.path.exists(INSTS_FILE):
        return out
    with open(INSTS_FILE) as f:
        for line in f:
            line = line.strip()
            if line.startswith("source_sha256:"):
                meta["sha"] = line.split(":", 1)[1].strip()
            elif line.startswith("pass "):
                head, tail = line.split(":", 1)
                _, prec, stage = head.split()
                kv = dict(t.split("=") for t in tail.split())
                out[f"{prec} {stage}"] = float(kv["valu_per_vn"])
    if meta.get("sha") != kernel_source_hash() or size != 4096:
        return {}
    return out


def copy_calibration(mib):
    """A plain device-to-device copy of known size (read mib MiB, write mib
    MiB), the reference for the HBM byte counters."""
    import torch

    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"bench: copy calibration, 3 copies of {mib} MiB ({mib * (1 << 20)} bytes read + written)")
    del src, dst
    torch.cuda.empty_cache()


def run_precision(I, W, N, storage, steps, warmup, seed, horizon=0, tau=1e-7):
    """Timed steps of the 2D workload in one storage type.  With horizon >
    warmup + steps the run then continues untimed to `horizon` steps and the
    moments at that horizon are returned as well."""
    import torch

    dt = 0.5 / N / PMAX8
    cfg = I.Config(d=2, nx=N, ny=N, q_phi=8, q_chi=8, K=2, tau=tau, dt=dt, storage=storage)
    states, k = W.quadrant_states(seed)
    fields = W.riemann_2d(N, N, states)
    s = I.Solver(cfg)
    s.set_equilibrium(*fields)
    if warmup:
        s.step(warmup)
    # the timed steps in up to 5 repetitions of equal length (HIP-event
    # time per step of each repetition reported beside the wall clock)
    nrep = min(5, steps) if steps > 0 else 1
    chunks = [steps // nrep + (1 if i < steps % nrep else 0) for i in range(nrep)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = [s.step_timed(c) for c in chunks]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = sum(reps)
    rep_each = [float(r.sum()) / c for r, c in zip(reps, chunks) if c > 0]
    rep_ms = sorted(rep_each)
    ok = s.check_state()
    cells = N * N
    planes = cfg.planes
    vn = cells * planes * steps / wall
    elem = 4 if storage == I.F32 else 8
    pb = pass_bytes(planes, cells, elem, 4)
    per = {k2: ms[i] / steps for i, k2 in enumerate(("stage3", "stage4", "stage5"))}
    step_bytes = sum(pb.values())
    res = {
        "value": vn,
        "ms_per_step": 1e3 * wall / steps,
        "ms_per_step_reps": {"median": rep_ms[len(rep_ms) // 2], "min": rep_ms[0], "max": rep_ms[-1],
                             "each": rep_each, "steps_each": chunks},
        "pass_ms": per,
        "pass_bytes": pb,
        "bytes_per_vn_step": step_bytes / (cells * planes),
        "step_gbs": step_bytes / (wall / steps) / 1e9,
        "state_ok": ok == I.OK,
        "seed_offset": k,
    }
    gbs4 = pb["stage4"] / (per["stage4"] * 1e-3) / 1e9
    prec = "f32" if elem == 4 else "f64"
    traffic = read_traffic(N).get(f"{prec} stage4")
    res["roofline"] = {"bound": "hbm", "kernel": "stage4 (stage2d_kernel<%s, 4>)" %
                       ("float" if elem == 4 else "double"),
                       "achieved": gbs4, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": gbs4 / HBM_PEAK_GBS, "traffic": traffic,
                       "algorithmic_bytes_per_launch": pb["stage4"],
                       "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                                       "copy-calibrated)"}
    # the VALU view of every pass: lane-instructions per VN (committed
    # counter summary) x VN / pass time, against the lane-slot peak
    vpv = read_valu_per_vn(N)
    if vpv:
        valu = {}
        for k2 in ("stage3", "stage4", "stage5"):
            rate = vpv[f"{prec} {k2}"] * cells * planes / (per[k2] * 1e-3) / 1e12
            valu[k2] = {"lane_insts_per_vn": vpv[f"{prec} {k2}"], "achieved": rate, "frac": rate / VALU_PEAK_T}
        res["roofline"]["valu"] = {"peak": VALU_PEAK_T, "unit": "T lane-instructions/s", "passes": valu,
                                   "source": "profiles/stage_passes_riemann4096_inst_mix.txt (SQ_INSTS_VALU)"}
        if valu["stage4"]["frac"] > res["roofline"]["frac"]:
            # the pass is closer to its VALU peak than to HBM: report that bound,
            # the HBM view beside it
            hbm = {key: res["roofline"][key] for key in ("achieved", "peak", "unit", "frac")}
            res["roofline"].update({"bound": "alu", "achieved": valu["stage4"]["achieved"], "peak": VALU_PEAK_T,
                                    "unit": "T lane-instructions/s", "frac": valu["stage4"]["frac"],
                                    "hbm": hbm})
    res["moments"] = s.moments()  # (n, ux, uy, T) after warmup + timed steps
    done = warmup + steps
    if horizon > done:
        t1 = time.perf_counter()
        while done < horizon:
            k = min(500, horizon - done)
            s.step(k)
            torch.cuda.synchronize()
            done += k
            log(f"bench: {N}^2 {'FP32' if elem == 4 else 'FP64'} at step {done} of {horizon}")
        res["horizon"] = {"steps": horizon, "moments": s.moments(), "state_ok": s.check_state() == I.OK,
                          "ms_per_step_after_timed": 1e3 * (time.perf_counter() - t1) / (horizon - warmup - steps)}
    del s
    torch.cuda.empty_cache()
    return res, cfg, fields


COPY_PROBE_BYTES = 4 << 30
CACHE_PROBE_BYTES = 64 << 20


def hbm_copy_rate(I, nbytes=COPY_PROBE_BYTES):
    """Achievable copy rate: best of 8 plain device copies of nbytes (GB/s,
    read plus written) by the library's copy probe; 4 GiB measures HBM,
    64 MiB (source and destination together inside the 256 MB last-level
    cache) the cache."""
    import torch

    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    gbs = I.copy_probe(src, dst, 8)
    del src, dst
    torch.cuda.empty_cache()
    return gbs


ALLOCATOR_WARMUP_BYTES = 64 << 30


def allocator_warmup():
    """Allocate and free one 64 GiB block before the workload's buffers.
    The FP64 stage-4 pass at 4096^2 runs at 13.6 ms on some allocations of
    its buffers and at 14.6 ms on others, for the life of the buffers; the
    first large allocation on a freshly started GPU has always been a slow
    one, and allocations after it mostly fast.  The block is never touched."""
    import torch

    try:
        x = torch.empty(ALLOCATOR_WARMUP_BYTES, dtype=torch.uint8, device="cuda")
    except RuntimeError as e:  # not enough free device memory: go on without it
        log(f"bench: allocator warm-up skipped ({e})")
        return 0
    torch.cuda.synchronize()
    del x
    torch.cuda.empty_cache()
    return ALLOCATOR_WARMUP_BYTES


def fp32_error(m32, m64):
    """Errors of the FP32-storage run against the FP64 run after the same
    steps: density and pressure relative (L1 over the grid and max), velocity
    absolute in units of c_ref."""
    import torch

    n32, ux32, uy32, T32 = m32
    n64, ux64, uy64, T64 = m64
    P32, P64 = n32 * T32, n64 * T64
    du = torch.sqrt((ux32 - ux64) ** 2 + (uy32 - uy64) ** 2)

    def rel(a, b):
        d = (a - b).abs()
        return {"l1_rel": float(d.sum() / b.abs().sum()), "max_rel": float(d.max() / b.abs().max())}

    return {"rho": rel(n32, n64), "P": rel(P32, P64),
            "u": {"l1_abs": float(du.mean()), "max_abs": float(du.max())}}


def horizon_1024(I, W, seed):
    """Configuration of the 1024^2 four-quadrant problem (tau 1e-6, CFL 0.5):
    FP64 and FP32 storage from the same seeded state to 500 steps; errors of
    the FP32-storage moments against the FP64 run at the end."""
    r64, _, _ = run_precision(I, W, 1024, I.F64, 10, 0, seed, horizon=500, tau=1e-6)
    r32, _, _ = run_precision(I, W, 1024, I.F32, 10, 0, seed, horizon=500, tau=1e-6)
    return {"workload": "1024x1024 four-quadrant problem, 8x8 velocities per f and g, tau 1e-6, "
                        "CFL 0.5, outflow",
            "steps": 500,
            "f64_ms_per_step": r64["horizon"]["ms_per_step_after_timed"],
            "f32_ms_per_step": r32["horizon"]["ms_per_step_after_timed"],
            "state_ok": r64["horizon"]["state_ok"] and r32["horizon"]["state_ok"],
            "error_vs_fp64": fp32_error(r32["horizon"]["moments"], r64["horizon"]["moments"])}


def host_cpu():
    """CPU model and logical CPU count of the host that runs the oracle."""
    model = "unknown CPU"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{model}, {os.cpu_count()} logical CPUs on the host"


MAX_ORACLE_THREADS = 16  # the host cores one GPU's share of the box provides


def oracle_threads():
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return max(1, min(MAX_ORACLE_THREADS, avail))


def cpu_baseline(O, W, cfg, fields, side, steps):
    """The FP64 oracle on side x side patches of the same workload: one
    patch at the quadrant corner on one core, then disjoint patches around it
    on all host cores at once (one independent oracle run per thread; each
    oracle call runs in C without the interpreter lock)."""
    import concurrent.futures as cf

    N = cfg.nx
    n, ux, uy, T = fields

    def patch_at(r0, c0):
        sl = (slice(r0, r0 + side), slice(c0, c0 + side))
        return tuple(np.ascontiguousarray(a[sl]) for a in (n, ux, uy, T))

    pc = O.Config(d=2, nx=side, ny=side, lx=side / N, ly=side / N, q_phi=8, q_chi=8, K=2,
                  tau=cfg.tau, dt=cfg.dt)
    c0 = N // 2 - side // 2
    patch = patch_at(c0, c0)
    F = O.equilibrium(pc, *patch)
    t0 = time.perf_counter()
    ref = O.step(pc, F, steps)
    dt1 = time.perf_counter() - t0
    vn1 = side * side * pc.planes * steps / dt1

    nthr = oracle_threads()
    k = int(np.ceil(np.sqrt(nthr)))
    base = N // 2 - (k * side) // 2
    origins = [(base + (i // k) * side, base + (i % k) * side) for i in range(nthr)]
    starts = [O.equilibrium(pc, *patch_at(r, c)) for r, c in origins]
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=nthr) as pool:
        list(pool.map(lambda F0: O.step(pc, F0, steps), starts))
    dtn = time.perf_counter() - t0
    vnn = nthr * side * side * pc.planes * steps / dtn
    return {"value": vnn, "unit": "VN/s", "cores": nthr, "kind": "oracle",
            "sample": f"{nthr} disjoint {side}x{side}-cell patches x 128 planes around the quadrant "
                      f"corner, {steps} IMEX step(s) each, one single-threaded C (-O2) oracle run per "
                      f"core at once, {dtn:.1f} s",
            "single_core": {"value": vn1, "unit": "VN/s", "cores": 1,
                            "sample": f"one {side}x{side} patch at the quadrant corner, {steps} IMEX "
                                      f"step(s), {dt1:.1f} s"},
            "host": host_cpu()}, (pc, patch, ref)


def oracle_patch_errors(I, O, pc, patch, ref, steps):
    """The oracle's patch problem run on the GPU in FP64 and with FP32
    storage, against the oracle after the same steps: density and pressure
    relative (L1 over the patch and max), velocity absolute."""
    on, oux, ouy, oT = O.moments(pc, ref)
    oP = on * oT

    def rel(a, b):
        d = np.abs(a - b)
        return {"l1_rel": float(d.sum() / np.abs(b).sum()), "max_rel": float(d.max() / np.abs(b).max())}

    out = {"sample": f"{pc.nx}x{pc.ny} patch of the workload (outflow edges), {steps} IMEX steps"}
    for storage, tag in ((I.F64, "f64"), (I.F32, "f32_storage")):
        c = I.Config(d=2, nx=pc.nx, ny=pc.ny, lx=pc.lx, ly=pc.ly, q_phi=pc.q_phi, q_chi=pc.q_chi, K=pc.K,
                     tau=pc.tau, dt=pc.dt, storage=storage)
        s = I.Solver(c)
        s.set_equilibrium(*patch)
        s.step(steps)
        n, ux, uy, T = (t.cpu().numpy() for t in s.moments())
        du = np.sqrt((ux - oux) ** 2 + (uy - ouy) ** 2)
        out[tag] = {"rho": rel(n, on), "P": rel(n * T, oP),
                    "u": {"l1_abs": float(du.mean()), "max_abs": float(du.max())}}
        del s
    return out


def _kernel_key(name):
    """("f64"|"f32", "stage3"|..) for a stage kernel name, else None."""
    if "stage2d_kernel<" not in name and "stage1d_kernel<" not in name:
        return None
    args = name.split("<", 1)[1].split(">")[0].split(",")
    prec = "f32" if args[0].strip() == "float" else "f64"
    return prec, "stage" + args[1].strip()


def summarize_stats(dirs, cmds):
    """Text summary of rocprofv3 --kernel-trace --stats CSVs."""
    rows = []
    for d in dirs:
        for f in glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True):
            with open(f) as fh:
                rows += list(csv.DictReader(fh))
    print("# rocprofv3 kernel statistics (per-kernel launch durations)")
    for c in cmds:
        print(f"# command: {c}")
    print(f"# kernel sources: source_sha256: {kernel_source_hash()}")
    print(f"{'kernel':64s} {'calls':>6s} {'avg_ms':>10s} {'min_ms':>10s} {'max_ms':>10s} {'total_ms':>10s}")
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        name = r["Name"].replace("imexlb::(anonymous namespace)::", "")
        if len(name) > 64:
            name = name[:61] + "..."
        print(f"{name:64s} {int(r['Calls']):6d} {float(r['AverageNs']) / 1e6:10.4f} "
              f"{float(r['MinNs']) / 1e6:10.4f} {float(r['MaxNs']) / 1e6:10.4f} "
              f"{float(r['TotalDurationNs']) / 1e6:10.3f}")


def _pmc_dispatches(d, counter):
    """{kernel name: [value of counter per dispatch]} from a --pmc run."""
    acc = {}
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] != counter:
                    continue
                per = acc.setdefault(r["Kernel_Name"], {})
                per[r["Dispatch_Id"]] = per.get(r["Dispatch_Id"], 0.0) + float(r["Counter_Value"])
    return {k: list(v.values()) for k, v in acc.items()}


def _calib(vals):
    """Mean counter value of the calibration copies: the copy dispatches of
    at least half the largest one (small runtime copies are left out)."""
    top = max(vals)
    big = [v for v in vals if v >= 0.5 * top]
    return sum(big) / len(big), len(big)


def summarize_pmc(fetch_dir, write_dir, copy_mib, size, cmds):
    """HBM traffic per launch of the stage passes from FETCH_SIZE and
    WRITE_SIZE runs (KiB per dispatch), each scaled by the same counter on a
    plain copy of copy_mib MiB."""
    fetch_d = _pmc_dispatches(fetch_dir, "FETCH_SIZE")
    write_d = _pmc_dispatches(write_dir, "WRITE_SIZE")
    cb = copy_mib * (1 << 20)
    # the runtime's copy kernel (torch copy_ of copy_mib MiB), not the
    # library's copy probe, which the same run launches on 4 GiB
    copies = [k for k in fetch_d if "copybuffer" in k.lower() and k in write_d]
    ck = max(copies, key=lambda k: max(fetch_d[k]))
    cf, nf = _calib(fetch_d[ck])
    cw, nw = _calib(write_d[ck])
    ff = cb / (cf * 1024.0)
    fw = cb / (cw * 1024.0)
    fetch = {k: sum(v) / len(v) for k, v in fetch_d.items()}
    write = {k: sum(v) / len(v) for k, v in write_d.items()}
    cells = size * size
    print("# HBM traffic of the stage passes, 2D Riemann workload, "
          f"{size}x{size} cells x 128 planes")
    for c in cmds:
        print(f"# command: {c}")
    print(f"source_sha256: {kernel_source_hash()}")
    print(f"size: {size}")
    print(f"copy_kernel: {ck[:90]}")
    print(f"copy_bytes: {cb}  copy_fetch_kib: {cf:.1f} (mean of {nf})  "
          f"copy_write_kib: {cw:.1f} (mean of {nw})")
    print(f"fetch_factor: {ff:.4f}  write_factor: {fw:.4f}")
    for k in sorted(fetch):
        key = _kernel_key(k)
        if key is None or k not in write:
            continue
        prec, stage = key
        t = fetch[k] * 1024.0 * ff + write[k] * 1024.0 * fw
        alg = pass_bytes(128, cells, 4 if prec == "f32" else 8, 4)[stage]
        print(f"pass {prec} {stage}: fetch_kib={fetch[k]:.1f} write_kib={write[k]:.1f} "
              f"traffic_bytes={t:.4e} algorithmic_bytes={alg:.4e} ratio={t / alg:.3f}")


INST_COUNTERS = ("SQ_WAVES", "SQ_INSTS_VALU", "SQ_INSTS_SALU", "SQ_INSTS_LDS", "SQ_INSTS_SMEM",
                 "SQ_INSTS_VMEM_RD", "SQ_INSTS_VMEM_WR", "SQ_INSTS_BRANCH", "GRBM_GUI_ACTIVE")


def summarize_insts(d, size, cmds):
    """Instruction mix of the stage passes from one --pmc run of
    INST_COUNTERS: lane-instructions per velocity node (wave instructions x
    64 / VN) and the VALU floor of each pass, one wave64 VALU instruction per
    4 cycles per SIMD on 1024 SIMDs at 2.4 GHz, against the dispatch time."""
    vals = {c: {} for c in INST_COUNTERS}
    span = {}
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for r in csv.DictReader(fh):
                c = r["Counter_Name"]
                if c not in vals:
                    continue
                key = (r["Kernel_Name"], r["Dispatch_Id"])
                vals[c][key] = vals[c].get(key, 0.0) + float(r["Counter_Value"])
                span[key] = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6
    vn = size * size * 128
    print("# Instruction mix of the stage passes, 2D Riemann workload, "
          f"{size}x{size} cells x 128 planes (one dispatch per pass and storage type)")
    for c in cmds:
        print(f"# command: {c}")
    print(f"source_sha256: {kernel_source_hash()}")
    print("# per_vn: wave instructions x 64 / velocity nodes; valu_floor_ms: SQ_INSTS_VALU x 4 cycles "
          "/ (1024 SIMDs x 2.4 GHz); valu_frac = valu_floor_ms / dispatch_ms; gui_clock_ghz: "
          "GRBM_GUI_ACTIVE (summed over the 8 XCDs) / 8 / dispatch time, the clock the pass ran at")
    rows = {}
    for (name, disp), v in vals["SQ_INSTS_VALU"].items():
        key = _kernel_key(name)
        if key is None:
            continue
        rows[key] = (name, disp)
    for key in sorted(rows):
        k = rows[key]
        g = {c: vals[c].get(k, float("nan")) for c in INST_COUNTERS}
        per = {c: g[c] * 64.0 / vn for c in INST_COUNTERS[1:-1]}
        floor_ms = g["SQ_INSTS_VALU"] * 4.0 / (1024 * 2.4e9) * 1e3
        print(f"pass {key[0]} {key[1]}: dispatch_ms={span[k]:.3f} waves={g['SQ_WAVES']:.0f} "
              + " ".join(f"{c[9:].lower()}_per_vn={per[c]:.2f}" for c in per)
              + f" gui_active_cycles={g['GRBM_GUI_ACTIVE']:.4e} "
              f"gui_clock_ghz={g['GRBM_GUI_ACTIVE'] / 8 / (span[k] * 1e6):.2f} "
              f"valu_floor_ms={floor_ms:.3f} valu_frac={floor_ms / span[k]:.3f}")


def batch_pass_bytes(vn, elem):
    """Algorithmic HBM bytes of the three 1D passes over vn velocity nodes
    (16 planes, 3 FP64 moment fields)."""
    m = 3 * 8 / 16.0
    return {"stage3": vn * (2 * elem + 2 * m), "stage4": vn * (4 * elem + 3 * m),
            "stage5": vn * (3 * elem + 2 * m)}


def run_batch(args, emit=True):
    """Batched 1D shock tubes: 256 seeded tubes of 256..4096 cells, K 0/2,
    tau 1e-6..1e-2, 8 + 8 velocities, FP32 storage, CFL 0.5 each.  Prints
    the JSON line (emit) and returns it as a dict."""
    import torch

    from paper_1909_08390_amd import imexlb as I
    from paper_1909_08390_amd import workloads as W

    tubes = W.batch_tubes(args.tubes, seed=args.seed, nx_range=tuple(args.tube_nx))
    specs = [I.TubeSpec(nx=t.nx, K=t.K, lx=1.0, tau=t.tau, dt=W.tube_dt(t.nx)) for t in tubes]
    storage = I.F64 if args.batch_f64 else I.F32
    b = I.Batch(specs, 8, 8, storage)
    f = [W.tube_fields(t) for t in tubes]
    b.set_equilibrium([x[0] for x in f], [x[1] for x in f], [x[2] for x in f])
    tune = b.tune(args.tune_steps)
    plan = b.plan()
    log(f"bench: batch tuner ms/step {tune}, chosen {plan}")
    if args.warmup:
        b.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms = b.step_timed(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n = b.moments()[0]
    ok = bool(torch.isfinite(n).all()) and float(n.min()) > 0
    cells = b.cells
    vn = cells * 16
    elem = 4 if storage == I.F32 else 8
    pb = batch_pass_bytes(vn, elem)
    step_ms = float(ms.sum()) / args.steps
    step_bytes = sum(pb.values())
    if plan.mode == 0:
        per = {k: ms[i] / args.steps for i, k in enumerate(("stage3", "stage4", "stage5"))}
        gbs4 = pb["stage4"] / (per["stage4"] * 1e-3) / 1e9
        rkernel, rbytes = "stage4 (stage1d_batch_kernel)", pb["stage4"]
    else:
        # one launch covers whole steps: the roofline of the persistent
        # kernel over a launch is the step's bytes over the step's time
        per = {"persistent_step": step_ms}
        gbs4 = step_bytes / (step_ms * 1e-3) / 1e9
        rkernel, rbytes = f"stage1d_persist_kernel ({plan.steps} steps per launch)", step_bytes * plan.steps
    value = vn * args.steps / wall
    best0 = min(v for k, v in tune.items() if k.mode == 0)
    best1 = min(v for k, v in tune.items() if k.mode == 1)
    cache_gbs = hbm_copy_rate(I, CACHE_PROBE_BYTES)
    log(f"bench: 64 MiB device copy (cache-resident) {cache_gbs:.0f} GB/s")
    cpu = None
    if not args.no_cpu:
        import oracle as O
        # the oracle on the first tubes of the batch until ~10 s of work
        done, vns, t_cpu, used = 0, 0, 0.0, []
        for t, sp in zip(tubes, specs):
            oc = O.Config(d=1, nx=t.nx, lx=1.0, q_phi=8, q_chi=8, K=t.K, tau=t.tau, dt=sp.dt)
            fn, fu, fT = W.tube_fields(t)
            F = O.equilibrium(oc, fn, fu, None, fT)
            c0 = time.perf_counter()
            O.step(oc, F, args.cpu_steps)
            t_cpu += time.perf_counter() - c0
            vns += t.nx * 16 * args.cpu_steps
            used.append(t.nx)
            done += 1
            if t_cpu > 10.0:
                break
        single = {"value": vns / t_cpu, "unit": "VN/s", "cores": 1,
                  "sample": f"first {done} tubes of the batch (nx {used}), {args.cpu_steps} IMEX "
                            f"steps each, single-threaded C (-O2), {t_cpu:.1f} s"}
        # every tube of the batch, one independent oracle run per tube, on
        # all host cores at once (each oracle call runs in C without the
        # interpreter lock)
        import concurrent.futures as cf

        def one(ts):
            t, sp = ts
            oc = O.Config(d=1, nx=t.nx, lx=1.0, q_phi=8, q_chi=8, K=t.K, tau=t.tau, dt=sp.dt)
            fn, fu, fT = W.tube_fields(t)
            O.step(oc, O.equilibrium(oc, fn, fu, None, fT), args.cpu_steps)

        nthr = oracle_threads()
        c0 = time.perf_counter()
        with cf.ThreadPoolExecutor(max_workers=nthr) as pool:
            list(pool.map(one, sorted(zip(tubes, specs), key=lambda ts: -ts[0].nx)))
        t_all = time.perf_counter() - c0
        cpu = {"value": cells * 16 * args.cpu_steps / t_all, "unit": "VN/s", "cores": nthr, "kind": "oracle",
               "sample": f"all {len(tubes)} tubes, {args.cpu_steps} IMEX steps each, one single-threaded C "
                         f"(-O2) oracle run per tube on {nthr} cores at once, {t_all:.1f} s",
               "single_core": single, "host": host_cpu()}
    out = {
        "metric": METRIC, "value": value, "unit": "VN/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * wall / args.steps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 storage, f64 moments" if elem == 4 else "f64",
        "data": "synthetic",
        "config": {"workload": f"{len(tubes)} batched 1D shock tubes, Nx {args.tube_nx[0]}..{args.tube_nx[1]} "
                               f"(sum {cells}), "
                               "K in {0,2}, tau 1e-6..1e-2, 8+8 velocities, CFL 0.5, outflow",
                   "cells": cells, "planes": 16, "seed": args.seed,
                   "plan": {"mode": "persistent" if plan.mode else "per-pass launches", "tile": plan.tile,
                            "order": plan.order, "chunk": plan.chunk, "steps_per_launch": plan.steps,
                            "bins": plan.bins},
                   "tuner_ms_per_step": {f"mode{k.mode} tile{k.tile} order{k.order} chunk{k.chunk} "
                                         f"steps{k.steps} bins{k.bins}": v for k, v in tune.items()},
                   "tuner_best_ms_per_step": {"per_pass_launches": best0, "persistent": best1}},
        "roofline": {"bound": "hbm", "kernel": rkernel, "achieved": gbs4,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs4 / HBM_PEAK_GBS,
                     "traffic": None, "algorithmic_bytes_per_launch": rbytes,
                     "note": "working set (~%.0f MB) fits the 256 MB last-level cache"
                             % ((b.state.numel() * elem * 3) / 1e6),
                     "cache_copy_gbs": cache_gbs, "frac_of_cache_copy": gbs4 / cache_gbs},
        "pass_ms": per,
        "state_ok": ok,
        "cpu_baseline": cpu,
    }
    if emit:
        print(json.dumps(out), flush=True)
    return out


def run_adjoint(args, emit=True):
    """Gradient of a density loss through a checkpointed rollout: 512^2
    periodic, 8 x 8 velocities per distribution, 200 steps, checkpoints every
    20 steps, FP32 storage; seeded Fourier density, u = 0, P = 1.  Prints
    the JSON line (emit) and returns it as a dict."""
    import torch

    from paper_1909_08390_amd import adjoint as A
    from paper_1909_08390_amd import imexlb as I
    from paper_1909_08390_amd import workloads as W

    N, steps, every = args.adj_size, args.adj_steps, 20
    dt = 0.5 / N / PMAX8
    cfg = I.Config(d=2, nx=N, ny=N, q_phi=8, q_chi=8, K=2, tau=1e-6, dt=dt, bc_x=I.PERIODIC,
                   bc_y=I.PERIODIC, storage=I.F32)
    s = I.Solver(cfg)
    n0 = torch.as_tensor(W.fourier_density(N, N, seed=args.seed), device="cuda")
    target = torch.as_tensor(W.fourier_density(N, N, seed=args.seed + 1), device="cuda")
    A.density_loss_gradient(s, n0, target, 2, every=every)  # warm-up
    torch.cuda.synchronize()
    zero = torch.zeros_like(n0)
    # forward-only rollouts and gradients interleaved, medians of three each
    # (a single forward of 200 steps lasts about 0.1 s, so one sample moves
    # with the clock state)
    t_fwds, t_grads = [], []
    for _ in range(3):
        t0 = time.perf_counter()
        s.set_equilibrium(n0, zero, zero, 1.0 / n0)
        s.step(steps)
        torch.cuda.synchronize()
        t_fwds.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        loss, grad = A.density_loss_gradient(s, n0, target, steps, every=every)
        torch.cuda.synchronize()
        t_grads.append(time.perf_counter() - t0)
    t_fwd, t_grad = float(np.median(t_fwds)), float(np.median(t_grads))
    vn = N * N * cfg.planes * steps
    cpu = None
    if not args.no_cpu:
        import oracle as O
        # the oracle's forward step (it has no adjoint) on a 64 x 64 patch of
        # the same periodic field, for context
        side, nst = 64, 4
        pc = O.Config(d=2, nx=side, ny=side, lx=side / N, ly=side / N, q_phi=8, q_chi=8, K=2, tau=cfg.tau,
                      dt=dt, bc_x=O.PERIODIC, bc_y=O.PERIODIC)
        nn = n0.cpu().numpy()[:side, :side].copy()
        z = np.zeros_like(nn)
        F = O.equilibrium(pc, nn, z, z, 1.0 / nn)
        c0 = time.perf_counter()
        O.step(pc, F, nst)
        t_cpu = time.perf_counter() - c0
        cpu = {"value": side * side * pc.planes * nst / t_cpu, "unit": "VN/s", "cores": 1, "kind": "oracle",
               "sample": f"forward only (the oracle has no adjoint): {side}x{side} periodic patch x 128 planes, "
                         f"{nst} IMEX steps, single-threaded C (-O2), {t_cpu:.1f} s", "host": host_cpu()}
    out = {
        "metric": "velocity-node updates/s per IMEX step, forward + adjoint (gradient)",
        "value": vn / t_grad, "unit": "VN/s", "n_gpus": 1, "steps": steps, "warmup": 1,
        "ms_per_step": 1e3 * t_grad / steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 storage (state and stage adjoints), f64 moments, lambda and arithmetic",
        "data": "synthetic",
        "config": {"workload": f"2D periodic {N}x{N}, 8x8 velocities per f and g, {steps} steps, "
                               f"checkpoint every {every}; loss 1/2 sum (n - n*)^2, gradient "
                               "w.r.t. the initial density (u = 0, P = 1)",
                   "cells": N * N, "planes": cfg.planes, "seed": args.seed},
        "forward_only_ms_per_step": 1e3 * t_fwd / steps,
        "gradient_over_forward": t_grad / t_fwd,
        "reps": {"forward_ms_per_step": [1e3 * t / steps for t in t_fwds],
                 "gradient_ms_per_step": [1e3 * t / steps for t in t_grads]},
        "loss": loss,
        "grad_norm": float(grad.norm()),
        "cpu_baseline": cpu,
    }
    if emit:
        print(json.dumps(out), flush=True)
    return out


def other_workloads(args):
    """The batched tubes and the gradient rollout, run briefly after the main
    workload so that the default bench line carries their measured rates
    (their own --workload runs give the full records)."""
    a = argparse.Namespace(**vars(args))
    a.no_cpu, a.steps, a.warmup = True, 20, 3
    log("bench: batched tubes (20 timed steps after the tuner)")
    rb = run_batch(a, emit=False)
    log(f"bench: batched tubes {rb['value']:.3e} VN/s, {rb['ms_per_step']:.3f} ms/step")
    log("bench: gradient through the 512^2 rollout")
    ra = run_adjoint(a, emit=False)
    log(f"bench: gradient {ra['ms_per_step']:.3f} ms/step, {ra['gradient_over_forward']:.2f}x the forward")
    return {
        "batch_tubes": {"value": rb["value"], "unit": "VN/s", "ms_per_step": rb["ms_per_step"],
                        "steps": a.steps, "dtype": rb["dtype"], "workload": rb["config"]["workload"],
                        "plan": rb["config"]["plan"], "tuner_best_ms_per_step": rb["config"]["tuner_best_ms_per_step"],
                        "roofline": {k: rb["roofline"][k] for k in ("kernel", "achieved", "peak", "unit", "frac",
                                                                      "cache_copy_gbs", "frac_of_cache_copy")}},
        "gradient_rollout": {"value": ra["value"], "unit": "VN/s", "ms_per_step": ra["ms_per_step"],
                             "steps": ra["steps"], "dtype": ra["dtype"], "workload": ra["config"]["workload"],
                             "forward_only_ms_per_step": ra["forward_only_ms_per_step"],
                             "gradient_over_forward": ra["gradient_over_forward"], "reps": ra["reps"]},
    }


def run_sod(args):
    """The paper's Sod tube: d = 1, 400 cells on [0, 1], 5 + 3 velocities,
    K = 2, tau = 1e-5, dt = 2.5e-4, the full 400 steps to t = 0.1, outflow.
    Three launches per step over 3,200 velocity nodes: launch-latency bound."""
    import torch

    from paper_1909_08390_amd import imexlb as I
    from paper_1909_08390_amd import workloads as W

    nx, nsteps = 400, 400
    cfg = I.Config(d=1, nx=nx, q_phi=5, q_chi=3, K=2, tau=1e-5, dt=2.5e-4)
    n, u, T = W.sod_1d(nx)
    s = I.Solver(cfg)
    s.set_equilibrium(n, u, None, T)
    s.step(args.warmup)
    s.set_equilibrium(n, u, None, T)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms = s.step_timed(nsteps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    vn = nx * cfg.planes * nsteps
    pb = {k: v for k, v in zip(("stage3", "stage4", "stage5"),
                               (nx * cfg.planes * (2 * 8 + 2 * 3 * 8 / cfg.planes),
                                nx * cfg.planes * (4 * 8 + 3 * 3 * 8 / cfg.planes),
                                nx * cfg.planes * (3 * 8 + 2 * 3 * 8 / cfg.planes)))}
    per = {k: ms[i] / nsteps for i, k in enumerate(("stage3", "stage4", "stage5"))}
    gbs4 = pb["stage4"] / (per["stage4"] * 1e-3) / 1e9
    # the same run without per-pass events, and as a batch of one tube under
    # the tuner's plan (persistent launches cover up to 8 steps each): the
    # step is launch-latency bound, so fewer launches is the lever
    s.set_equilibrium(n, u, None, T)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.step(nsteps)
    torch.cuda.synchronize()
    wall_plain = time.perf_counter() - t0
    ref = s.state.clone()
    b = I.Batch([I.TubeSpec(nx=nx, K=2, tau=1e-5, dt=2.5e-4)], q_phi=5, q_chi=3, storage=I.F64)
    b.set_equilibrium(n, u, T)
    tuned = b.tune(8)
    b.set_equilibrium(n, u, T)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(nsteps)
    torch.cuda.synchronize()
    wall_batch = time.perf_counter() - t0
    plan = b.plan()
    one_tube = {"us_per_step": 1e6 * wall_batch / nsteps, "value": vn / wall_batch, "unit": "VN/s",
                "plan": {"mode": "persistent launches" if plan.mode == 1 else "per-pass launches",
                         "tile": plan.tile, "steps_per_launch": plan.steps, "bins": plan.bins},
                "tuner_best_us_per_step": {
                    "per_pass_launches": 1e3 * min(v for k, v in tuned.items() if k.mode == 0),
                    "persistent": 1e3 * min(v for k, v in tuned.items() if k.mode == 1)},
                "state_bitwise_equal_to_single_grid": bool(torch.equal(b.tube_state(0), ref))}
    cpu = None
    if not args.no_cpu:
        import oracle as O
        oc = O.Config(d=1, nx=nx, q_phi=5, q_chi=3, K=2, tau=1e-5, dt=2.5e-4)
        F = O.equilibrium(oc, n, u, None, T)
        c0 = time.perf_counter()
        O.step(oc, F, nsteps)
        t_cpu = time.perf_counter() - c0
        cpu = {"value": vn / t_cpu, "unit": "VN/s", "cores": 1, "kind": "oracle",
               "sample": f"the whole run ({nsteps} IMEX steps), single-threaded C (-O2), {t_cpu:.2f} s",
               "host": host_cpu()}
    out = {
        "metric": METRIC, "value": vn / wall, "unit": "VN/s", "n_gpus": 1, "steps": nsteps,
        "warmup": args.warmup, "ms_per_step": 1e3 * wall / nsteps, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "Sod shock tube, 400 cells on [0,1], 5+3 velocities, K=2 (gamma 7/5), "
                               "tau=1e-5, dt=2.5e-4, 400 steps to t=0.1, outflow",
                   "cells": nx, "planes": cfg.planes},
        "us_per_step": 1e6 * wall / nsteps,
        "us_per_step_without_pass_events": 1e6 * wall_plain / nsteps,
        "one_tube_batch": one_tube,
        "pass_ms": per,
        "roofline": {"bound": "hbm", "kernel": "stage4 (stage1d_kernel<double, 4>)", "achieved": gbs4,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs4 / HBM_PEAK_GBS, "traffic": None,
                     "algorithmic_bytes_per_launch": pb["stage4"],
                     "note": "3,200 velocity nodes per pass: bound by launch latency, not by HBM"},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def run_slab(args):
    """One GPU's share of the 4096^2 workload split into y-slabs: the step on
    a 4096 x (4096 / slabs) slab at the full problem's cell size and time step
    (the slab through the quadrant corner, outflow rows standing in for the
    neighbours' halos), FP64 and FP32 storage, and the halo bytes a sharded
    step would exchange per pass.  No multi-GPU path exists in this library;
    the exchange time is an estimate from the xGMI link rate, not measured."""
    import torch

    from paper_1909_08390_amd import imexlb as I
    from paper_1909_08390_amd import workloads as W

    N, parts = args.size, args.slabs
    ny = N // parts
    ly = ny / N
    dt = 0.5 / N / PMAX8
    states, k = W.quadrant_states(args.seed)
    res = {}
    for storage, name in ((I.F64, "f64"), (I.F32, "f32")):
        cfg = I.Config(d=2, nx=N, ny=ny, lx=1.0, ly=ly, q_phi=8, q_chi=8, K=2, tau=1e-7, dt=dt,
                       storage=storage)
        s = I.Solver(cfg)
        s.set_equilibrium(*W.riemann_2d(N, ny, states, x0=0.5, y0=0.5 * ly, lx=1.0, ly=ly))
        s.step(args.warmup)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ms = s.step_timed(args.steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        elem = 4 if storage == I.F32 else 8
        res[name] = {"ms_per_step": 1e3 * wall / args.steps, "value": N * ny * cfg.planes * args.steps / wall,
                     "unit": "VN/s",
                     "pass_ms": {kk: ms[i] / args.steps for i, kk in enumerate(("stage3", "stage4", "stage5"))},
                     # per pass and side: 5 ghost rows of the pass's stencil input and of its moments
                     "halo_bytes_per_pass_per_side": 5 * N * (cfg.planes * elem + 4 * 8)}
        res[name]["halo_ms_per_step_one_link_estimate"] = (
            3 * 2 * res[name]["halo_bytes_per_pass_per_side"] / (XGMI_LINK_GBS * 1e9) * 1e3)
        del s
        torch.cuda.empty_cache()
    out = {
        "metric": METRIC, "value": res["f64"]["value"], "unit": "VN/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": res["f64"]["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"one of {parts} y-slabs of the {N}x{N} four-quadrant problem: {N}x{ny} cells, "
                               "8x8 velocities per f and g, tau=1e-7, the full problem's dt, outflow",
                   "cells": N * ny, "planes": 128, "seed": args.seed + k},
        "slab": res,
        "xgmi_link_gbs_assumed": XGMI_LINK_GBS,
        "note": "single-GPU share only; the halo exchange is not implemented, its time is bytes / one link's rate",
    }
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size", type=int, default=4096)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--horizon", type=int, default=2000,
                    help="after the timed steps, continue both storage types to this many steps "
                         "and report the FP32-vs-FP64 errors there (and at 500 steps of the 1024^2 "
                         "problem); 0 skips")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-side", type=int, default=128)
    ap.add_argument("--cpu-steps", type=int, default=10)
    ap.add_argument("--copy-calib", type=int, default=0, metavar="MIB",
                    help="first run a plain copy of MIB MiB (counter calibration)")
    ap.add_argument("--summarize-stats", nargs="+", metavar="DIR",
                    help="print a summary of rocprofv3 --stats CSVs and exit")
    ap.add_argument("--summarize-pmc", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="print the HBM traffic summary of two --pmc runs and exit")
    ap.add_argument("--summarize-insts", metavar="DIR",
                    help="print the instruction-mix summary of a --pmc run of INST_COUNTERS and exit")
    ap.add_argument("--cmd", action="append", default=[],
                    help="command line recorded in a summary")
    ap.add_argument("--slabs", type=int, default=8, help="slab workload: y-slabs of the grid")
    ap.add_argument("--workload", choices=["riemann2d", "batch", "adjoint", "sod", "slab"], default="riemann2d",
                    help="riemann2d: the 4096^2 2D step (default); batch: 256 1D tubes; "
                         "adjoint: gradient through a 512^2 rollout; sod: the paper's 400-cell tube")
    ap.add_argument("--adj-size", type=int, default=512)
    ap.add_argument("--adj-steps", type=int, default=200)
    ap.add_argument("--tubes", type=int, default=256)
    ap.add_argument("--batch-f64", action="store_true")
    ap.add_argument("--tube-nx", type=int, nargs=2, default=[256, 4096], metavar=("LO", "HI"),
                    help="range of the batched tubes' cell counts")
    ap.add_argument("--tune-steps", type=int, default=8,
                    help="steps per plan timed by the batch autotuner")
    ap.add_argument("--no-others", action="store_true",
                    help="skip the short batched-tube and gradient runs of the default workload")
    args = ap.parse_args()

    if args.summarize_stats:
        summarize_stats(args.summarize_stats, args.cmd)
        return
    if args.summarize_insts:
        summarize_insts(args.summarize_insts, args.size, args.cmd)
        return
    if args.summarize_pmc:
        summarize_pmc(args.summarize_pmc[0], args.summarize_pmc[1], args.copy_calib, args.size,
                      args.cmd)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only; multi-GPU figures are not "
              "part of it (the sharding design is described in DESIGN.md).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1909_08390_amd import imexlb as I
    from paper_1909_08390_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    warm = allocator_warmup()
    if args.copy_calib:
        copy_calibration(args.copy_calib)
    if args.workload == "batch":
        run_batch(args)
        return
    if args.workload == "adjoint":
        run_adjoint(args)
        return
    if args.workload == "sod":
        run_sod(args)
        return
    if args.workload == "slab":
        run_slab(args)
        return
    horizon = args.horizon if args.horizon > args.warmup + args.steps else 0
    log(f"bench: {args.size}^2 cells x 128 planes, FP64, {args.warmup} warmup + {args.steps} steps"
        + (f", then on to step {horizon}" if horizon else ""))
    r64, cfg, fields = run_precision(I, W, args.size, I.F64, args.steps, args.warmup, args.seed, horizon)
    log(f"bench: FP64 {r64['value']:.3e} VN/s, {r64['ms_per_step']:.2f} ms/step, passes {r64['pass_ms']}")
    r32 = None
    if not args.no_fp32:
        log("bench: FP32 storage run")
        r32, _, _ = run_precision(I, W, args.size, I.F32, args.steps, args.warmup, args.seed, horizon)
        log(f"bench: FP32 {r32['value']:.3e} VN/s, {r32['ms_per_step']:.2f} ms/step, passes {r32['pass_ms']}")
    h1024 = None
    if not args.no_fp32 and args.horizon > 0 and args.size == 4096:
        log("bench: 1024^2 FP32-vs-FP64 run to 500 steps")
        h1024 = horizon_1024(I, W, args.seed)
        log(f"bench: 1024^2 after 500 steps: {h1024['error_vs_fp64']}")
    copy_gbs = hbm_copy_rate(I)
    log(f"bench: plain device copy {copy_gbs:.0f} GB/s")
    others = None if args.no_others else other_workloads(args)
    cpu = patch_err = None
    if not args.no_cpu:
        import oracle as O
        log("bench: CPU oracle baseline")
        cpu, (pc, patch, ref) = cpu_baseline(O, W, cfg, fields, args.cpu_side, args.cpu_steps)
        log(f"bench: oracle {cpu['value']:.3e} VN/s")
        patch_err = oracle_patch_errors(I, O, pc, patch, ref, args.cpu_steps)
        log(f"bench: GPU vs oracle on the patch: {patch_err}")

    out = {
        "metric": METRIC,
        "value": r64["value"],
        "unit": "VN/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"2D four-quadrant Riemann problem, {args.size}x{args.size} cells, "
                        "8x8 Gauss-Hermite velocities per f and g (128 planes), K=2 "
                        "(gamma 7/5), tau=1e-7, CFL 0.5, outflow",
            "cells": args.size * args.size, "planes": 128, "dt": cfg.dt,
            "seed": args.seed + r64["seed_offset"],
        },
        "roofline": r64["roofline"],
        "pass_ms": r64["pass_ms"],
        "ms_per_step_reps": r64["ms_per_step_reps"],
        "bytes_per_vn_step": r64["bytes_per_vn_step"],
        "step_hbm_frac": r64["step_gbs"] / HBM_PEAK_GBS,
        "allocator_warmup_bytes": warm,
        "hbm_copy": {"gbs": copy_gbs, "frac_of_peak": copy_gbs / HBM_PEAK_GBS,
                     "bytes": COPY_PROBE_BYTES, "reps": 8,
                     "kernel": "imexlb_copy_probe: one 16-byte load and store per thread",
                     "stage4_frac_of_copy": r64["roofline"]["achieved"] / copy_gbs,
                     "step_frac_of_copy": r64["step_gbs"] / copy_gbs},
        "cpu_baseline": cpu,
        "error_vs_oracle": patch_err,
        "other_workloads": others,
    }
    if r32 is not None:
        err = fp32_error(r32["moments"], r64["moments"])
        log(f"bench: FP32 vs FP64 after {args.warmup + args.steps} steps: {err}")
        out["fp32"] = {
            "value": r32["value"], "unit": "VN/s", "dtype": "f32 storage, f64 moments",
            "ms_per_step": r32["ms_per_step"], "pass_ms": r32["pass_ms"],
            "ms_per_step_reps": r32["ms_per_step_reps"],
            "speedup_vs_fp64": r32["value"] / r64["value"],
            "bytes_per_vn_step": r32["bytes_per_vn_step"],
            "step_hbm_frac": r32["step_gbs"] / HBM_PEAK_GBS,
            "roofline": r32["roofline"],
            "error_vs_fp64": err,
            "error_after_steps": args.warmup + args.steps,
        }
        if horizon and "horizon" in r32 and "horizon" in r64:
            herr = fp32_error(r32["horizon"]["moments"], r64["horizon"]["moments"])
            log(f"bench: FP32 vs FP64 after {horizon} steps: {herr}")
            out["fp32"]["horizons"] = [
                {"workload": f"{args.size}x{args.size} (this bench's workload)", "steps": horizon,
                 "f64_ms_per_step": r64["horizon"]["ms_per_step_after_timed"],
                 "f32_ms_per_step": r32["horizon"]["ms_per_step_after_timed"],
                 "state_ok": r64["horizon"]["state_ok"] and r32["horizon"]["state_ok"],
                 "error_vs_fp64": herr}]
            if h1024 is not None:
                out["fp32"]["horizons"].append(h1024)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
