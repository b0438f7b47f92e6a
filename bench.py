"""Benchmark of the fused ideal-MHD step on one MI355X.

Workload: 3D periodic decaying MHD turbulence on a 512^3 grid, FP32 state
and arithmetic (FP64 CFL reduction and conservation sums), PLM minmod +
HLLD + GLM, SSP-RK2, CFL 0.3; synthetic seeded initial fields.

A timed step is one pass of the whole hot path: the CFL maxima of the
previous step's output are read back (one 16-byte device-to-host copy and
stream sync), the GLM decay factor is formed, and mhd_step runs both stage
kernels with the fused ghost fill, reconstruction, Riemann fluxes, flux
divergence, psi damping, CFL and FP64-sum reductions.  Inputs are resident
in HBM before timing starts.

Prints one JSON line with the throughput (Mcell-updates/s), the HBM
roofline of the dominant kernel (stage 2: algorithmic bytes per launch over
its average duration from HIP events recorded on the library's stream,
against 8 TB/s), beside it the VALU issue roof that binds that kernel, FP64
figures on the same workload, the paper's benchmark scheme
(WENO-Z + HLLD + GLM + SSP-RK3) on its two problems (3D Orszag-Tang, 3D
circularly polarised Alfven wave) at the per-GPU share 416^3, the
adjoint/forward time ratio, and the FP64 CPU oracle timed on a bounded
sample of the workload as a baseline.
"""
import argparse
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
VALU_PEAK_TLANE = 1024 * 16 * 2.4e9 / 1e12  # 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
METRIC = "Mcell-updates/s + % HBM roofline (FP32 vs FP64), adjoint/forward time ratio"


def _code_only(text):
    """C++ source without comments and blank lines (string literals kept)."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c == '"':
            j = i + 1
            while j < n and text[j] != '"':
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    return "\n".join(ln.rstrip() for ln in "".join(out).splitlines() if ln.strip())


def kernel_source_hash():
    """Hash of the kernel sources' code (comments and blank lines do not
    count: the stored counters stay valid across comment edits)."""
    h = hashlib.sha256()
    for p in sorted(glob.glob(os.path.join(ROOT, "paper_2510_24175_amd", "csrc", "*"))):
        with open(p, encoding="utf-8") as f:
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def measured_counters(kernel_key):
    """rocprofv3 counter figures of one kernel launch (HBM bytes, VALU
    instructions), if the stored measurement was taken on the current kernel
    sources; None otherwise."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    ent = data.get(kernel_key)
    if not isinstance(ent, dict) or ent.get("source_hash") != kernel_source_hash():
        return None
    return ent


def run_gpu(n, dtype, steps, warmup, workload="turbulence", limiter="minmod", time_order=2, **gen_args):
    import torch

    from paper_2510_24175_amd import workloads
    from paper_2510_24175_amd.mhd import Context

    setup, V = getattr(workloads, workload)(n, **gen_args)
    setup["limiter"], setup["time_order"] = limiter, time_order
    ctx = Context(setup, dtype)
    Vd = torch.from_numpy(V).cuda()
    del V
    a = ctx.prim_to_cons(Vd)
    del Vd
    b = torch.empty_like(a)
    ncell = n * n * n

    def one_step(first):
        nonlocal a, b
        if first:
            dt, ch = ctx.cfl_dt(a)
        else:
            dt, ch, _ = ctx.step_info()
        ctx.step(a, b, dt, ch, ctx.damp(dt, ch))
        a, b = b, a

    first = True
    for _ in range(warmup):
        one_step(first)
        first = False
    torch.cuda.synchronize()
    ctx.timing_start(steps)
    t0 = time.perf_counter()
    for _ in range(steps):
        one_step(first)
        first = False
    _, _, sums = ctx.step_info()  # includes the last step's completion
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    nt, st1, st2, red = ctx.timing_stop()
    # the same steps with dt and c_h held at the last values (no per-step
    # read-back and host synchronisation): what the CFL read-back costs
    dt, ch, _ = ctx.step_info()
    dmp = ctx.damp(dt, ch)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(steps):
        ctx.step(a, b, dt, ch, dmp)
        a, b = b, a
    torch.cuda.synchronize()
    wall_fixed = time.perf_counter() - t1
    s = 4 if dtype == "f32" else 8
    res = {
        "ms_per_step_fixed_dt": 1e3 * wall_fixed / steps,
        "ms_per_step": 1e3 * wall / steps,
        "mcells": ncell * steps / wall / 1e6,
        "stage1_ms": st1 / nt,
        "stage2_ms": st2 / nt,
        "reduce_ms": red / nt,
        "elem": s,
        "ncell": ncell,
        "sums": sums,
    }
    # algorithmic HBM traffic: the first stage reads Un and writes U1
    # (18 s B/cell), every later stage reads Un and its input stage and
    # writes its output (27 s B/cell): 45 s B/cell per SSP-RK2 step, 72 s
    # per SSP-RK3 step.  Constrained transport, per stage: the stage kernel
    # reads the input's 9 components and 3 faces (and Un's 9 after the first
    # stage) and writes 6 components and 6 transverse fluxes (24 s | 33 s);
    # the EMF pass reads 6 fluxes and writes 3 EMFs (9 s); the face pass
    # reads 3 EMFs and the input's 3 faces (and Un's 3 after the first
    # stage), writes 3 faces and 3 cell-field components, and in the last
    # stage reads 6 components for the reductions (12 s | 15 s | 21 s):
    # 45 s, 57 s and 63 s B/cell for the first, a middle and the last stage.
    # With the upwind EMF the stage kernel writes no fluxes (18 s | 27 s) and
    # the EMF pass reads the input's 8 cell and 3 face components and writes
    # 3 EMFs (14 s): 44 s, 56 s and 62 s.
    if setup.get("ct", False):
        if setup.get("ct_emf") == "upwind":
            stages = [44] + [56] * (time_order - 2) + [62]
        else:
            stages = [45] + [57] * (time_order - 2) + [63]
        res["alg_bytes_step"] = sum(stages) * s * ncell
    else:
        res["alg_bytes_step"] = (18 + 27 * (time_order - 1)) * s * ncell
    res["alg_bytes_stage2"] = 27 * s * ncell
    res["hbm_frac_step"] = res["alg_bytes_step"] / (wall / steps) / (HBM_PEAK_GBS * 1e9)
    del a, b
    ctx.close()
    torch.cuda.empty_cache()
    return res


def run_adjoint_ratio(n, dtype, steps):
    """Time mhd_step (forward) and mhd_step_adjoint (given the stage-1
    state) on the same state in the same way: each loop of `steps` calls is
    enqueued without host synchronisation (dt, c_h and the decay factor held
    fixed) and bracketed by events on the stream the library enqueues on
    (torch's current stream)."""
    import torch

    from paper_2510_24175_amd import workloads
    from paper_2510_24175_amd.mhd import Context

    setup, V = workloads.turbulence(n)
    ctx = Context(setup, dtype, adjoint=True)
    a = ctx.prim_to_cons(torch.from_numpy(V).cuda())
    del V
    b = torch.empty_like(a)
    u1 = torch.empty_like(a)
    dt, ch = ctx.cfl_dt(a)
    dmp = ctx.damp(dt, ch)
    lam = torch.randn(a.shape, dtype=torch.float64, device="cuda") * 1e-3
    lam_n = torch.empty_like(lam)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    for _ in range(2):  # warm-up
        ctx.step(a, b, dt, ch, dmp, U1_out=u1)
        ctx.step_adjoint(a, u1, lam, lam_n, dt, ch, dmp)
    ctx.step_info()
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(steps):
        ctx.step(a, b, dt, ch, dmp, U1_out=u1)
    ev[1].record()
    ev[2].record()
    for _ in range(steps):
        ctx.step_adjoint(a, u1, lam, lam_n, dt, ch, dmp)
    ev[3].record()
    torch.cuda.synchronize()
    ctx.step_info()  # raises if either loop met a non-physical state
    fwd = ev[0].elapsed_time(ev[1]) / steps
    adj = ev[2].elapsed_time(ev[3]) / steps
    ctx.close()
    del a, b, u1, lam, lam_n
    torch.cuda.empty_cache()
    return {"n": n, "dtype": dtype, "forward_ms": round(fwd, 4), "adjoint_ms": round(adj, 4),
            "ratio": round(adj / fwd, 3), "target": 3.0, "meets_target": bool(adj / fwd <= 3.0),
            "backward_incl_recompute_ratio": round((adj + fwd) / fwd, 3)}


def copy_bandwidth(mib=2048, reps=5):
    """Achievable HBM bandwidth: a plain device-to-device copy of MIB MiB
    (read + write bytes per copy over its event-timed duration)."""
    import torch

    a = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del a, b
    return 2 * (mib << 20) / (ms * 1e-3) / 1e9


def cpu_model():
    """The host CPU's model name as lscpu reports it (else /proc/cpuinfo)."""
    import subprocess
    try:
        txt = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for ln in txt.splitlines():
            if ln.strip().startswith("Model name:"):
                return ln.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    try:
        with open("/proc/cpuinfo") as f:
            return next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), None)
    except OSError:
        return None


def _oracle_rate(workload, n, steps, threads):
    """Mcell-updates/s of the FP64 oracle over `steps` full steps (CFL
    included) of a workload generator at size n on `threads` host threads;
    returns (rate, wall seconds, threads used)."""
    from oracle import coracle
    from paper_2510_24175_amd import workloads

    coracle.set_threads(threads)
    setup, V = getattr(workloads, workload)(n)
    o = coracle.Oracle(setup)
    U = o.prim_to_cons(V)
    ncell = setup["n"][0] * setup["n"][1] * setup["n"][2]
    t0 = time.perf_counter()
    done = 0
    t = 0.0
    t_end = setup.get("t_end")
    while done < steps and not (t_end is not None and t >= t_end * (1 - 1e-14)):
        dt, ch = o.cfl(U)
        if t_end is not None and t + dt > t_end:
            dt = t_end - t
        U = o.step(U, dt, ch)
        t += dt
        done += 1
    wall = time.perf_counter() - t0
    return ncell * done / wall / 1e6, wall, coracle.threads(), done


def cpu_baseline(n_sample=256, steps=4, n_single=64, steps_single=4):
    """FP64 CPU oracle on a bounded sample of the same workload: the same
    turbulence generator (modes, spectra, amplitudes) on an n_sample^3
    periodic grid, stepped with the same scheme on all host threads (about
    10 s of host work), and on an n_single^3 grid on one thread."""
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    rate, wall, used, _ = _oracle_rate("turbulence", n_sample, steps, threads)
    rate1, wall1, _, _ = _oracle_rate("turbulence", n_single, steps_single, 1)
    return {
        "value": round(rate, 3),
        "unit": "Mcell-updates/s",
        "cores": used,
        "cpu_model": cpu_model(),
        "kind": "oracle",
        "sample": f"turbulence {n_sample}^3 (same generator, FP64, PLM minmod + HLLD + GLM), "
                  f"{steps} full RK2 steps incl. CFL, {wall:.1f} s wall on {used} threads",
        "single_thread": {"value": round(rate1, 3), "unit": "Mcell-updates/s", "cores": 1,
                          "sample": f"turbulence {n_single}^3, {steps_single} steps, {wall1:.1f} s wall"},
    }


def cpu_configs(threads):
    """The FP64 oracle on the small configurations: Brio-Wu 400 cells to
    t = 0.1 (complete), turbulence 128^3 for 100 steps, the 1024^2
    Orszag-Tang vortex for a bounded number of steps (the rate; the full run
    to t = 0.5 takes some 9000 steps), on all host threads and on one
    thread (bounded step counts there)."""
    rows = []
    for workload, n, steps_all, steps_one in [("brio_wu", 400, 10 ** 6, 10 ** 6),
                                              ("turbulence", 128, 100, 3),
                                              ("orszag_tang", 1024, 100, 5)]:
        for thr, steps in ((threads, steps_all), (1, steps_one)):
            rate, wall, used, done = _oracle_rate(workload, n, steps, thr)
            rows.append({"workload": workload, "n": n, "steps": done, "threads": used,
                         "wall_s": round(wall, 2), "mcell_updates_per_s": round(rate, 4)})
            print(json.dumps(rows[-1]), file=sys.stderr, flush=True)
    return {"cpu_model": cpu_model(), "oracle_configs": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-paper-scheme", action="store_true")
    ap.add_argument("--paper-n", type=int, default=416)
    ap.add_argument("--paper-cases", default="ot3d_f64,ot3d_f32,cpa3d_f64",
                    help="comma list of paper-scheme runs (ot3d_f64, ot3d_f32, cpa3d_f64, cpa3d_f32)")
    ap.add_argument("--no-ct", action="store_true")
    ap.add_argument("--ct-n", type=int, default=352)
    ap.add_argument("--ct-cases", default="f64,f32,f64_upwind",
                    help="comma list of constrained-transport runs: f64, f32 (mean edge EMF), "
                         "f64_upwind, f32_upwind (upwind edge EMF)")
    ap.add_argument("--cpu-configs", action="store_true",
                    help="only time the FP64 CPU oracle on the small configurations (no GPU)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB three times (counter calibration)")
    args = ap.parse_args()
    if args.cpu_configs:
        print(json.dumps(cpu_configs(int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)))))
        return
    if args.copy_probe:
        import torch
        a = torch.ones(args.copy_probe * (1 << 18), dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": a.numel() * 4}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)

    r32 = run_gpu(args.n, "f32", args.steps, args.warmup)
    print(f"# f32 {args.n}^3: {r32['ms_per_step']:.3f} ms/step, stage1 {r32['stage1_ms']:.3f} ms, "
          f"stage2 {r32['stage2_ms']:.3f} ms, reduce {r32['reduce_ms']:.3f} ms", file=sys.stderr,
          flush=True)
    out = {
        "metric": METRIC,
        "value": round(r32["mcells"], 2),
        "unit": "Mcell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r32["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": f"3D periodic decaying MHD turbulence {args.n}^3, FP32 state, FP64 CFL and sums, "
                        "PLM minmod + HLLD + GLM, SSP-RK2, CFL 0.3",
            "n": [args.n] * 3,
            "parallelism": "single GPU",
        },
    }
    # the roofline of the dominant kernel (stage 2): its algorithmic HBM
    # bytes per launch (27 s per cell: reads Un and U1, writes U_next) over
    # its event-timed average launch duration, against 8 TB/s
    ach = r32["alg_bytes_stage2"] / (r32["stage2_ms"] * 1e-3) / 1e9
    cnt = measured_counters(f"stage2_turbulence{args.n}_f32")
    traffic = cnt.get("bytes_per_launch") if cnt else None
    cgbs = copy_bandwidth()
    out["roofline"] = {
        "bound": "hbm",
        "kernel": "stage_kernel<float, HLLD, 3D, stage 2>",
        "achieved": round(ach, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(ach / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        "alg_bytes_per_launch": r32["alg_bytes_stage2"],
        "avg_launch_ms": round(r32["stage2_ms"], 4),
        "copy_gbs": round(cgbs, 1),
        "frac_of_copy": round(ach / cgbs, 4),
        "target_frac": 0.6,
        "meets_target": bool(ach / HBM_PEAK_GBS >= 0.6),
    }
    if cnt and cnt.get("valu_wave_insts"):
        # what binds the kernel instead: VALU issue.  Its VALU lane
        # instructions per launch (SQ_INSTS_VALU x 64, counted on these
        # sources) over the launch duration, against 1024 SIMDs x 16 lanes at
        # 2.4 GHz (a wave64 instruction occupies a SIMD for 4 cycles)
        lane_insts = cnt["valu_wave_insts"] * 64
        alu = lane_insts / (r32["stage2_ms"] * 1e-3) / 1e12
        out["alu_roofline"] = {
            "bound": "alu",
            "kernel": "stage_kernel<float, HLLD, 3D, stage 2>",
            "achieved": round(alu, 3),
            "peak": round(VALU_PEAK_TLANE, 3),
            "unit": "T VALU lane-instructions/s",
            "frac": round(alu / VALU_PEAK_TLANE, 4),
            "per_cell": round(lane_insts / r32["ncell"], 1),
        }
    out["hbm_frac_step_algorithmic"] = round(r32["hbm_frac_step"], 4)
    out["stage_ms"] = {"stage1": round(r32["stage1_ms"], 4), "stage2": round(r32["stage2_ms"], 4),
                       "final_reduce": round(r32["reduce_ms"], 4)}
    out["ms_per_step_fixed_dt"] = round(r32["ms_per_step_fixed_dt"], 4)
    if not args.no_fp64:
        r64 = run_gpu(args.n, "f64", max(3, args.steps // 2), 2)
        out["fp64"] = {
            "value": round(r64["mcells"], 2),
            "ms_per_step": round(r64["ms_per_step"], 4),
            "hbm_frac_step_algorithmic": round(r64["hbm_frac_step"], 4),
            "stage2_ms": round(r64["stage2_ms"], 4),
        }
    if not args.no_paper_scheme:
        # the scheme of the paper's benchmark runs (WENO-Z + HLLD + SSP-RK3,
        # GLM in the strong-scaling runs, double precision) on the per-GPU
        # share of the 832 x 832 x 416 strong-scaling grid split over one
        # node's four GPUs (416^3), for the paper's two problems: the 3D
        # Orszag-Tang vortex (FP64 and FP32) and the 3D circularly polarised
        # Alfven wave (FP64)
        pn = args.paper_n
        ps = {"workload": f"3D Orszag-Tang vortex and 3D circularly polarised Alfven wave, {pn}^3, "
                          "WENO-Z + HLLD + GLM, SSP-RK3, CFL 0.3", "n": [pn] * 3}
        cases = [c.strip() for c in args.paper_cases.split(",") if c.strip()]
        for key in cases:
            wl = {"ot3d": "orszag_tang_3d", "cpa3d": "cpa_wave_3d"}[key.split("_")[0]]
            dt_ = key.split("_")[1]
            r = run_gpu(pn, dt_, max(3, args.steps // 2), 2, workload=wl, limiter="wenoz", time_order=3)
            ach = r["alg_bytes_stage2"] / (r["stage2_ms"] * 1e-3) / 1e9
            ps[key] = {"value": round(r["mcells"], 2), "unit": "Mcell-updates/s",
                       "ms_per_step": round(r["ms_per_step"], 4),
                       "hbm_frac_step_algorithmic": round(r["hbm_frac_step"], 4),
                       "stage_ms": {"first_two": round(r["stage1_ms"], 4), "last": round(r["stage2_ms"], 4),
                                    "final_reduce": round(r["reduce_ms"], 4)},
                       "last_stage_gbs": round(ach, 1)}
            cnt = measured_counters(f"stage3_{wl}{pn}_{dt_}_wenoz_rk3")
            if cnt and cnt.get("valu_wave_insts"):
                ps[key]["last_stage_valu_issue_frac"] = round(
                    cnt["valu_wave_insts"] * 4 / (1024 * 2.4e9 * r["stage2_ms"] * 1e-3), 4)
            print(f"# paper scheme {key} {pn}^3: {r['ms_per_step']:.3f} ms/step", file=sys.stderr, flush=True)
        out["paper_scheme"] = ps
    if not args.no_ct:
        # the paper's weak-scaling runs: the same scheme with constrained
        # transport instead of GLM on its per-GPU share (704 x 704 x 352 per
        # four-GPU node, 352^3), 3D Orszag-Tang vortex
        cn = args.ct_n
        cs = {"workload": f"3D Orszag-Tang vortex {cn}^3, WENO-Z + HLLD, constrained transport (mean edge "
                          "EMF; _upwind: the upwind EMF), SSP-RK3, CFL 0.3", "n": [cn] * 3}
        for key in [c.strip() for c in args.ct_cases.split(",") if c.strip()]:
            dt_, _, emf = key.partition("_")
            r = run_gpu(cn, dt_, max(3, args.steps // 2), 2, workload="orszag_tang_3d_ct", limiter="wenoz",
                        time_order=3, emf=emf or "mean")
            cs[key] = {"value": round(r["mcells"], 2), "unit": "Mcell-updates/s",
                       "ms_per_step": round(r["ms_per_step"], 4),
                       "hbm_frac_step_algorithmic": round(r["hbm_frac_step"], 4),
                       "stage_ms": {"first_two": round(r["stage1_ms"], 4), "last": round(r["stage2_ms"], 4),
                                    "final_reduce": round(r["reduce_ms"], 4)}}
            print(f"# constrained transport {key} {cn}^3: {r['ms_per_step']:.3f} ms/step", file=sys.stderr,
                  flush=True)
        out["constrained_transport"] = cs
    if not args.no_adjoint:
        # adjoint/forward time ratio at the adjoint workload (128^3 FP32)
        # and at the benchmark grid
        out["adjoint"] = [run_adjoint_ratio(128, "f32", 10), run_adjoint_ratio(args.n, "f32", 3)]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
