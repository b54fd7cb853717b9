"""Benchmark of the colour-gradient D3Q19 step on one MI355X.

Workload: the 256^3 periodic emulsion (radii U[6,12], RSA to volume fraction
0.30, tau = 0.8, A = 0.005, beta = 0.7, near-contact strength 0.02 over 2
sites), seeded and synthetic.  A step is one full update of every site.

Prints ONE JSON line: MLUPS of the FP32-storage stepper (the headline value),
the same workload in the 16-bit storage forms, the roofline figures of the
dominant kernel (algorithmic bytes per launch over its HIP-event duration),
and the FP64 CPU oracle timed on this host as the CPU baseline.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# algorithmic bytes per site update, read + write: raw storage 2 components x
# 19 populations; 16-bit moment-split storage a 32-byte FP32 record plus 19
# 16-bit deviations per site (the plain 16-bit form of the same state would
# be 2 x 19 x 2 x 2 = 152 B)
ALGO_BYTES = {0: 2 * 19 * 2 * 8, 1: 2 * 19 * 2 * 4, 2: 2 * (32 + 19 * 2), 3: 2 * (32 + 19 * 2)}
STORE_NAME = {0: "f64", 1: "f32", 2: "f16", 3: "bf16"}


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def gpu_variant(w, storage, steps, warmup, stream, kernel=0):
    import torch
    from paper_2005_12764_amd import lb

    p = dict(w.params, storage=storage, kernel=kernel)
    L = lb.Lattice(p, stream=stream)
    try:
        L.init(w.rho_r, w.rho_b)
        L.step(warmup)
        torch.cuda.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        start.record(stream)
        L.step(steps)
        stop.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        ms = start.elapsed_time(stop) / steps
        # per-pass durations with HIP events on the lattice's stream
        k_ms = lb.lb_step_timed(L.h, min(steps, 50))
        tot = L.totals()
        ok = tot[6].sum() == 0 and np.isfinite(tot[:5].sum())
        return dict(ms_per_step=ms, wall_s=wall, kernel=L.kernel, pass_ms=k_ms, finite=bool(ok))
    finally:
        L.close()


def measured_traffic(label, n):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    summary (profiles/hbm_traffic_emulsion256.txt), or None when the kernel
    sources have changed since the counters were taken or the lattice is not
    the profiled 256^3 one."""
    import glob
    import hashlib
    path = os.path.join(ROOT, "profiles", "hbm_traffic_emulsion256.txt")
    if n != 256 or not os.path.exists(path):
        return None
    table = {}
    for line in open(path):
        if line.strip() and not line.startswith("#"):
            k, v = line.split()
            table[k] = v
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2005_12764_amd", "csrc")
    for src in sorted(glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.hpp"))):
        h.update(open(src, "rb").read())
    if table.get("sources") != h.hexdigest()[:16] or label not in table:
        return None
    return float(table[label])


def copy_bandwidth(stream, gib=2.0, reps=10):
    """Achievable HBM bandwidth of a plain device-to-device copy (read +
    write bytes per second), the practical ceiling next to the 8 TB/s peak."""
    import torch
    n = int(gib * 2 ** 30) // 4
    a = torch.empty(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    b.copy_(a)
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    best = float("inf")
    # the runtime's copy and torch's vectorised elementwise kernel; the faster counts
    for op in (lambda: b.copy_(a), lambda: torch.mul(a, 1.0, out=b)):
        op()
        start.record(stream)
        for _ in range(reps):
            op()
        stop.record(stream)
        torch.cuda.synchronize()
        best = min(best, start.elapsed_time(stop) / reps)
    ms = best
    del a, b
    torch.cuda.empty_cache()
    return 2 * n * 4 / (ms * 1e-3) / 1e9


def serving(reqs, prep, rate, steps, budget_gb, storage="f16"):
    import copy
    import torch
    from paper_2005_12764_amd import serve as S
    from paper_2005_12764_amd import workloads as W
    st = {"f32": W.F32, "f16": W.F16, "bf16": W.BF16}[storage]
    reqs = copy.deepcopy(reqs)
    for r in reqs:
        r.params = dict(r.params, storage=st)
    sstream = torch.cuda.Stream()
    be = S.GpuBackend(int(budget_gb * 2 ** 30), max_jobs=512, storage=st, chunk=50, stream=sstream)
    with torch.cuda.stream(sstream):
        rep = S.Server(be, chunk=50).run(reqs)
    be.close()
    out = rep.summary()
    out.update(storage=storage, rate_jobs_per_s=rate, steps_per_job=steps, budget_gb=budget_gb,
               request_prep_s=round(prep, 2))
    return out


def structure_factor(phi):
    """Shell-averaged |FFT(phi - <phi>)|^2 (torch FFT of a device field):
    returns (k, S(k)), the first moment k1 and the peak height."""
    import torch
    f = torch.fft.fftn(phi - phi.mean())
    p = (f.real ** 2 + f.imag ** 2)
    n = phi.shape[0]
    k1d = torch.fft.fftfreq(n, d=1.0 / n).to(phi.device)
    kz, ky, kx = torch.meshgrid(k1d, k1d, k1d, indexing="ij")
    kk = torch.sqrt(kx ** 2 + ky ** 2 + kz ** 2).round().long().flatten()
    nb = n // 2
    m = kk <= nb
    S = torch.zeros(nb + 1, dtype=torch.float64, device=phi.device).index_add_(0, kk[m], p.flatten()[m].double())
    cnt = torch.zeros(nb + 1, dtype=torch.float64, device=phi.device).index_add_(
        0, kk[m], torch.ones_like(p.flatten()[m], dtype=torch.float64))
    S = (S / cnt.clamp(min=1)).cpu().numpy()
    k = np.arange(nb + 1) * 2 * np.pi / n
    k1 = float((k[1:] * S[1:]).sum() / S[1:].sum())
    return k, S, k1, float(S[1:].max())


def config_c3(args, stream):
    """Microfluidic-crystal channel: FP32 and 16-bit storage against FP64."""
    from paper_2005_12764_amd import lb
    from paper_2005_12764_amd import workloads as W
    import torch
    w = W.crystal_channel(seed=0, steps=args.c_steps or 2000)
    res, states = {}, {}
    for name, st in (("f64", 0), ("f32", 1), ("f16", 2), ("bf16", 3)):
        # one |G| threshold for all storages, so that every run follows the same dynamics
        with lb.Lattice(dict(w.params, storage=st, eps_g=1e-6), stream=stream) as L:
            L.init(w.rho_r, w.rho_b)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            L.step(w.steps)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            states[name] = (L.state(),) + tuple(L.moments())
        res[name] = {"mlups": round(w.sites * w.steps / dt / 1e6, 1)}
        log("c3 %s: %.0f MLUPS" % (name, res[name]["mlups"]))

    def rel(a, b):
        return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))

    ref = states["f64"]
    for name in ("f32", "f16", "bf16"):
        f, rr, rb, j = states[name]
        e = {"populations": max(rel(f[k, i], ref[0][k, i]) for k in range(2) for i in range(19)),
             "rho_r": rel(rr, ref[1]), "rho_b": rel(rb, ref[2]),
             "momentum": float(np.linalg.norm((j - ref[3]).ravel())
                               / (np.sqrt(1 / 3) * np.linalg.norm((ref[1] + ref[2]).ravel()))),
             "max_abs": float(np.abs(f - ref[0]).max())}
        res[name]["err_vs_f64"] = {k: float("%.3e" % v) for k, v in e.items()}
    return {"config": "microfluidic crystal channel 512x128x64, walls y/z, force 1e-6, 138 droplets R=10",
            "steps": w.steps, "results": res}


def config_c4(args, stream):
    """Spinodal decomposition: structure factor of 16-bit storage vs FP32."""
    from paper_2005_12764_amd import lb
    from paper_2005_12764_amd import workloads as W
    import torch
    n = args.c4_n
    w = W.spinodal(seed=0, n=n)
    marks = [m for m in (1000, 2000, 5000) if m <= (args.c_steps or 5000)]
    res = {}
    for name, st in (("f32", 1), ("f16", 2), ("bf16", 3)):
        out = {}
        with lb.Lattice(dict(w.params, storage=st), stream=stream) as L:
            L.init(w.rho_r, w.rho_b)
            done, busy = 0, 0.0
            rr = torch.empty(w.shape, dtype=torch.float32, device="cuda")
            rb = torch.empty_like(rr)
            for m in marks:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                L.step(m - done)
                torch.cuda.synchronize()
                busy += time.perf_counter() - t0
                done = m
                lb.lb_moments(L.h, rr, rb, None)
                torch.cuda.synchronize()
                phi = ((rr - rb) / (rr + rb)).double()
                _, S, k1, peak = structure_factor(phi)
                out[m] = {"k1": k1, "peak": peak}
        res[name] = {"mlups": round(w.sites * done / busy / 1e6, 1), "S": out}
        log("c4 %s: %.0f MLUPS %s" % (name, res[name]["mlups"], out))
    for name in ("f16", "bf16"):
        for m in marks:
            a, b = res[name]["S"][m], res["f32"]["S"][m]
            a["k1_rel_err"] = abs(a["k1"] / b["k1"] - 1)
            a["peak_rel_err"] = abs(a["peak"] / b["peak"] - 1)
    return {"config": "spinodal %d^3 50/50, noise 0.01, tau 1, A 0.01, near-contact 0.03 over 2 sites" % n,
            "steps": marks[-1], "results": res}


def korteweg_leg(w, stream, b=4, reps=20):
    """The Korteweg-tensor diagnostic on the FP32 lattice of the workload: phase
    field of the state, K at every site, block averages over b^3 (device outputs)."""
    import torch
    from paper_2005_12764_amd import lb

    L = lb.Lattice(dict(w.params, storage=1), stream=stream)
    try:
        L.init(w.rho_r, w.rho_b)
        L.step(2)
        nz, ny, nx = w.shape
        K = torch.empty((6, nz // b, ny // b, nx // b), dtype=torch.float32, device="cuda")
        P = torch.empty((nz // b, ny // b, nx // b), dtype=torch.float32, device="cuda")
        lb.lb_korteweg(L.h, 1.0, b, K, P)
        torch.cuda.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        start.record(stream)
        for _ in range(reps):
            lb.lb_korteweg(L.h, 1.0, b, K, P)
        stop.record(stream)
        torch.cuda.synchronize()
        ms = start.elapsed_time(stop) / reps
        ok = bool(torch.isfinite(K).all().item() and torch.isfinite(P).all().item())
        return {"b": b, "ms_per_call": round(ms, 4), "mlups": round(w.sites / (ms * 1e-3) / 1e6, 1),
                "finite": ok, "field": "phase field of the one-read FP32 state (face-site assembly + tensor-and-block kernel)"}
    finally:
        L.close()


def cpu_baseline(w, steps, steps_1t):
    from oracle import oracle as O

    prm = O.params_from_dict(dict(w.params, storage=0))
    f = O.init(prm, w.rho_r, w.rho_b)
    t0 = time.perf_counter()
    O.step(prm, f, steps)
    dt = time.perf_counter() - t0
    cores = O.threads()
    out = dict(value=w.sites * steps / dt / 1e6, unit="MLUPS", cores=cores, kind="oracle",
               sample="%d step(s) of the full %s lattice (%d sites), FP64, OpenMP over sites"
                      % (steps, "x".join(str(s) for s in w.shape[::-1]), w.sites),
               seconds=dt)
    if steps_1t > 0:
        # the same oracle on one thread (a per-core figure)
        O.set_threads(1)
        try:
            t0 = time.perf_counter()
            O.step(prm, f, steps_1t)
            dt1 = time.perf_counter() - t0
        finally:
            O.set_threads(cores)
        out.update(value_1thread=w.sites * steps_1t / dt1 / 1e6, steps_1thread=steps_1t, seconds_1thread=dt1)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256, help="lattice side of the emulsion")
    ap.add_argument("--variants", default="f32,f16,bf16")
    ap.add_argument("--kernel", type=int, default=0, help="0 auto, 1 two-pass, 2 fused")
    ap.add_argument("--cpu-steps", type=int, default=20,
                    help="oracle steps of the full lattice on all host threads (about 35 s on 16)")
    ap.add_argument("--cpu-steps-1t", type=int, default=1, help="oracle steps on one thread (0 = skip)")
    ap.add_argument("--serve-jobs", type=int, default=200, help="jobs of the serving leg (0 = skip)")
    ap.add_argument("--serve-rate", type=float, default=40.0,
                    help="arrival rate of the serving leg (the design-sweep stream's 40 jobs/s)")
    ap.add_argument("--serve-sat-rate", type=float, default=1000.0,
                    help="arrival rate of a second serving leg that keeps the batch full "
                         "(its aggregate rate measures the serving form's capacity; 0 = skip)")
    ap.add_argument("--serve-steps", type=int, default=500)
    ap.add_argument("--serve-sat-storages", default="f32,bf16",
                    help="other storage forms the batch-kept-full stream also runs in, to set the "
                         "fp16 serving form beside them on the same jobs ('' = none)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-korteweg", action="store_true", help="skip the Korteweg-diagnostic leg")
    ap.add_argument("--config", default="c2", help="c2 (headline), c3 (crystal channel), c4 (spinodal)")
    ap.add_argument("--c-steps", type=int, default=0, help="steps of the c3/c4 runs (0 = the config's)")
    ap.add_argument("--c4-n", type=int, default=384)
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the domain decomposition is a design note); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    from paper_2005_12764_amd import workloads as W

    if args.config in ("c3", "c4"):
        import torch
        torch.cuda.set_device(0)
        stream = torch.cuda.current_stream()
        out = config_c3(args, stream) if args.config == "c3" else config_c4(args, stream)
        print(json.dumps(out), flush=True)
        return

    # the serving leg's requests (droplet lists) are built by worker
    # processes before this process touches the GPU
    reqs, prep, sat_reqs = None, 0.0, None
    if args.serve_jobs > 0:
        from paper_2005_12764_amd import serve as S
        t0 = time.perf_counter()
        reqs = S.make_requests(args.serve_jobs, seed=0, rate=args.serve_rate, steps=args.serve_steps)
        if args.serve_sat_rate > 0:
            sat_reqs = S.make_requests(args.serve_jobs, seed=0, rate=args.serve_sat_rate, steps=args.serve_steps)
        prep = time.perf_counter() - t0
        log("serving: %d requests prepared in %.1fs" % (len(reqs), prep))

    import torch
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    w = W.periodic_emulsion(seed=0, n=args.n, storage=W.F32)
    log("workload %s: %d sites, %d droplets, phi_v %.3f (%.1fs)"
        % (w.name, w.sites, w.info["n_droplets"], w.info["rsa_phi_v"], time.perf_counter() - t0))

    codes = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}
    results = {}
    for name in args.variants.split(","):
        st = codes[name]
        r = gpu_variant(w, st, args.steps, args.warmup, stream, args.kernel)
        r["mlups"] = w.sites / (r["ms_per_step"] * 1e-3) / 1e6
        r["algo_gbs"] = r["mlups"] * 1e6 * ALGO_BYTES[st] / 1e9
        # the tile kernel alone (pass_ms[1]) against its algorithmic bytes
        r["tile_algo_gbs"] = ALGO_BYTES[st] * w.sites / (r["pass_ms"][1] * 1e-3) / 1e9
        results[name] = r
        log("%s: %.3f ms/step, %.0f MLUPS, %.0f GB/s algorithmic, passes %s"
            % (name, r["ms_per_step"], r["mlups"], r["algo_gbs"], r["pass_ms"]))

    head = results.get("f32") or next(iter(results.values()))
    head_name = "f32" if "f32" in results else next(iter(results))
    st = codes[head_name]
    # dominant kernel: the collide-and-stream pass (pass_ms[1]; pass_ms[0] is the
    # phase pass of two-pass steps or the phase assembly of one-read steps)
    dom_ms = head["pass_ms"][1]
    achieved = ALGO_BYTES[st] * w.sites / (dom_ms * 1e-3) / 1e9
    traffic = measured_traffic("collide_" + head_name, args.n)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": None if traffic is None else round(traffic / 1e9, 3),
            "traffic_unit": "GB per launch (rocprofv3 FETCH_SIZE x2 + WRITE_SIZE)",
            "kernel": ("collide pass (z-marching fused_kernel, phase field from the phase pass)"
                       if head["kernel"] == 1 else
                       "one-read tile (lean_kernel; face-site phase field completed by assemble_kernel)"),
            "algo_bytes_per_site": ALGO_BYTES[st], "sites_per_launch": w.sites,
            "kernel_ms": round(dom_ms, 4)}

    copy_gbs = copy_bandwidth(stream)
    log("device copy: %.0f GB/s (read + write)" % copy_gbs)
    roof["copy_gbs"] = round(copy_gbs, 1)
    roof["frac_of_copy"] = round(achieved / copy_gbs, 4)
    if head_name == "f32" and head["kernel"] == 2:
        # the same kernel's memory access pattern without its arithmetic
        # (lb_pattern_ms): the ceiling of that pattern on this device
        from paper_2005_12764_amd import lb
        pat_ms = lb.lb_pattern_ms(dict(w.params, storage=W.F32), 20)
        pat_gbs = ALGO_BYTES[st] * w.sites / (pat_ms * 1e-3) / 1e9
        log("one-read access pattern without arithmetic: %.3f ms, %.0f GB/s" % (pat_ms, pat_gbs))
        roof["pattern_gbs"] = round(pat_gbs, 1)
        roof["frac_of_pattern"] = round(achieved / pat_gbs, 4)

    kort = None
    if not args.no_korteweg:
        kort = korteweg_leg(w, stream)
        log("korteweg: %s" % kort)

    serve_out = sat_out = None
    sat_by = {}
    if args.serve_jobs > 0:
        serve_out = serving(reqs, prep, args.serve_rate, args.serve_steps, 0.8 * 288)
        log("serving: %s" % serve_out)
        if sat_reqs is not None:
            sat_out = serving(sat_reqs, prep, args.serve_sat_rate, args.serve_steps, 0.8 * 288)
            log("serving, batch kept full: %s" % sat_out)
            for name in filter(None, args.serve_sat_storages.split(",")):
                o = serving(sat_reqs, prep, args.serve_sat_rate, args.serve_steps, 0.8 * 288, storage=name)
                log("serving, batch kept full, %s storage: %s" % (name, o))
                sat_by[name] = {k: o[k] for k in ("aggregate_mlups", "device_mlups", "p50_s", "p99_s")}

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(w, args.cpu_steps, args.cpu_steps_1t)
        log("cpu oracle: %.2f MLUPS on %d threads (%.1fs)" % (cpu["value"], cpu["cores"], cpu["seconds"]))
        if "value_1thread" in cpu:
            log("cpu oracle: %.3f MLUPS on 1 thread (%.1fs)" % (cpu["value_1thread"], cpu["seconds_1thread"]))

    out = {
        "metric": "MLUPS and HBM GB/s (% of peak), FP16-store vs FP32; p50/p99 sweep-job latency",
        "value": round(head["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "periodic emulsion %d^3, phi_v 0.30, R U[6,12], tau 0.8, A 0.005, "
                               "beta 0.7, near-contact 0.02 over 2 sites" % args.n,
                   "sites": w.sites, "storage": head_name,
                   "kernel": "two-pass" if head["kernel"] == 1 else "one-read",
                   "parallelism": "single GPU"},
        "hbm_gbs_algorithmic": round(head["algo_gbs"], 1),
        "hbm_frac_algorithmic": round(head["algo_gbs"] / HBM_PEAK_GBS, 4),
        "variants": {k: {"mlups": round(v["mlups"], 1), "ms_per_step": round(v["ms_per_step"], 4),
                         "algo_gbs": round(v["algo_gbs"], 1),
                         "pass_ms": [round(x, 4) for x in v["pass_ms"]],
                         "tile_algo_gbs": round(v["tile_algo_gbs"], 1),
                         "finite": v["finite"]} for k, v in results.items()},
        "roofline": roof,
        "korteweg": kort,
        "serving": serve_out,
        "serving_saturated": sat_out,
        "serving_saturated_other_storage": sat_by or None,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
