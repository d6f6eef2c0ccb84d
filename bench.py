"""Throughput of the HEALPix SHT hot path on one MI355X.

One step = forward (map2alm) + inverse (alm2map) transform of a batch of B
maps resident in HBM.  Default workload: Nside=1024 (12,582,912 pixels),
lmax=2047, B=16 FP32 channels of band-limited Gaussian random fields with
C_l = (l+10)^-2.

Prints one JSON line: maps/s, per-step p50/p99 latency, the roofline of the
dominant kernel (timed with HIP events recorded on the transform's stream
inside the timed region) and the FP64 CPU oracle's rate on a bounded sample.
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {  # MI355X published peaks
    "hbm_GBs": 8000.0,
    "fp32_vector_TFs": 157.3,
    "fp64_vector_TFs": 78.6,
    "fp32_mfma_TFs": 157.3,
    "fp64_mfma_TFs": 78.6,
    "bf16_mfma_TFs": 2500.0,
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--nside", type=int, default=1024)
    ap.add_argument("--lmax", type=int, default=None)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64", "bf16"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="sht", choices=["sht", "serving", "jacobi", "reorder", "resize", "grad", "nested"],
                    help="sht: forward+inverse throughput (default); serving: Poisson trace of mixed "
                         "requests through the serving loop vs one at a time; jacobi: 3-iteration "
                         "refined analysis at Nside=2048, lmax=4095, one map; reorder: RING <-> NESTED "
                         "pixel order conversion of --batch maps at --nside; resize: spectral resize of "
                         "--batch coefficient sets from lmax 2 nside - 1 to 4 nside - 1; grad: forward + "
                         "spectral loss + adjoint backward at --nside, --batch, --dtype; nested: analysis of "
                         "NESTED maps, fused layout conversion vs nest2ring + map2alm")
    ap.add_argument("--stored-lambda", action="store_true",
                    help="with --dtype bf16: also time the forward with the resident stored-lambda table")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--rate", type=float, default=200.0)
    ap.add_argument("--budget-gib", type=float, default=48.0)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--merge-channels", type=int, default=64,
                    help="serving: merge queued requests of one geometry into calls of up to this many "
                         "channels (0: every request its own call)")
    ap.add_argument("--peaks", action="store_true",
                    help="only measure the device's HBM copy bandwidth and GEMM (matrix-core) rates "
                         "with torch library calls, print one JSON line and exit")
    ap.add_argument("--calibrate-copy-mib", type=int, default=0,
                    help="only run a plain device copy of this many MiB (5 times), "
                         "to calibrate HBM byte counters, and exit")
    return ap.parse_args()


# Legendre kernels: the library takes the matrix-core kernels for FP32 /
# BF16 contraction and for FP64 from this many channels up (its default
# switch points), the vector-ALU kernels otherwise
MFMA_MIN_BATCH = {"fwd": 5, "inv": 8}
MFMA64_MIN_BATCH = {"fwd": 3, "inv": 5}


def on_mfma(stage, dtype, batch):
    d = stage.split("_")[1]
    if dtype == "f64":
        return batch >= MFMA64_MIN_BATCH[d]
    return dtype in ("f32", "bf16") and batch >= MFMA_MIN_BATCH[d]


def bf16_mfma(stage, dtype, batch):
    """BF16 maps take the BF16 matrix-core analysis from the FP32 switch point."""
    return stage == "legendre_fwd" and dtype == "bf16" and batch >= MFMA_MIN_BATCH["fwd"]


def stage_kernel(stage, dtype, batch):
    """(kernel symbol, source file) that runs `stage`."""
    if bf16_mfma(stage, dtype, batch):
        return ("k_legendre_fwd_bf16", "legendre_bf16.hip")
    if stage == "pack_bf16":
        return ("k_pack_spectra_bf16", "legendre_bf16.hip")
    if stage.startswith("legendre"):
        d = stage.split("_")[1]
        if not on_mfma(stage, dtype, batch):
            return ("k_legendre_%s_valu" % d, "legendre_valu.hip")
        return ("k_legendre_%s_mfma64" % d, "legendre_mfma64.hip") if dtype == "f64" else \
            ("k_legendre_%s_mfma" % d, "legendre_mfma.hip")
    return {"ring_fft_fwd": ("k_ring_fft_fwd", "ring_fft.hip"),
            "ring_fft_inv": ("k_ring_fft_inv", "ring_fft.hip"),
            "alm_in": ("k_alm_in", "layout.hip")}[stage]


def source_sha(fname):
    path = os.path.join(ROOT, "paper_2510_01785_amd", "csrc", fname)
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(kernel, fname, workload):
    """HBM bytes per dispatch of `kernel` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE, calibrated on a plain copy), or None when the
    summary is missing or the kernel source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_%s.txt" % workload)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        text = f.read()
    m = re.search(r"^%s\s+source=(\w+)\s+fetch_bytes=([0-9.e+]+)\s+write_bytes=([0-9.e+]+)" % kernel,
                  text, re.M)
    if not m or m.group(1) != source_sha(fname):
        return None
    return float(m.group(2)) + float(m.group(3))


def rel_l2(got, ref):
    return float(np.linalg.norm((got - ref).ravel()) / max(np.linalg.norm(ref.ravel()), 1e-300))


def per_l_max_rel(got, ref, lmax):
    """max over l of |a_l. - ref_l.| / |ref_l.| (norms over m = 0..l), and its l."""
    from paper_2510_01785_amd import synth
    ls, _ = synth.lm_arrays(lmax)
    num = np.bincount(ls, weights=np.abs(got - ref) ** 2, minlength=lmax + 1)
    den = np.bincount(ls, weights=np.abs(ref) ** 2, minlength=lmax + 1)
    r = np.sqrt(num / np.maximum(den, 1e-300))
    return float(r.max()), int(r.argmax())


def oracle_check(nside, lmax, f0, a0_gpu, g0_gpu):
    """The FP64 oracle, as it stands, on channel 0 of the timed step: its
    forward transform of the timed input map f0 and its inverse transform of
    the step's own coefficients a0_gpu.  Timed (forward + inverse, all host
    threads) as the CPU baseline, and compared element by element with the
    step's outputs (a0_gpu, and g0_gpu = the step's synthesis of a0_gpu, or
    None for a forward-only step): relative l2 and the largest per-l relative
    error of the coefficients, relative l2 of the map, and the round-trip
    error f0 - S(A(f0)) of the GPU path (RMS and max, relative to f0)."""
    from oracle import _clib, sht
    _clib.build()
    t0 = time.perf_counter()
    a_ref = sht.map2alm(f0[None, :], lmax, nside)[0]
    g_ref = sht.alm2map(a0_gpu[None, :].astype(np.complex128), nside, lmax)[0]
    dt = time.perf_counter() - t0
    acc = {"map2alm_rel_l2": float("%.3e" % rel_l2(a0_gpu, a_ref))}
    worst, lw = per_l_max_rel(a0_gpu, a_ref, lmax)
    acc["map2alm_per_l_max_rel"] = float("%.3e" % worst)
    acc["map2alm_per_l_max_at_l"] = lw
    if g0_gpu is not None:
        acc["alm2map_rel_l2"] = float("%.3e" % rel_l2(g0_gpu, g_ref))
        d = f0 - g0_gpu
        acc["round_trip_rms_rel"] = float("%.3e" % (np.sqrt(np.mean(d ** 2)) / np.sqrt(np.mean(f0 ** 2))))
        acc["round_trip_max_rel"] = float("%.3e" % (np.abs(d).max() / np.abs(f0).max()))
    acc["oracle"] = "FP64 CPU oracle on channel 0 of the timed step"
    cpu = dict(value=round(1.0 / dt, 5), unit="maps/s", cores=_clib.threads(), kind="oracle",
               sample="channel 0 of the timed step (nside=%d, lmax=%d): oracle forward of its input map "
                      "+ inverse of its coefficients, %.1f s" % (nside, lmax, dt))
    return acc, cpu


def stage_peak(bound, dtype):
    """Peak (flop/s or B/s) of a stage's bound: the matrix cores of the
    contraction's precision (FP32, or FP64 at the FP64 rate; BF16 maps on
    the FP32 contraction count as FP32), the vector ALUs of the compute
    precision otherwise."""
    if bound == "hbm":
        return PEAK["hbm_GBs"] * 1e9
    if bound == "mfma":
        return (PEAK["fp64_mfma_TFs"] if dtype == "f64" else PEAK["fp32_mfma_TFs"]) * 1e12
    return (PEAK["fp64_vector_TFs"] if dtype == "f64" else PEAK["fp32_vector_TFs"]) * 1e12


def step_roofline(stages, work, dtype, B, ms_per_step):
    """Roofline time of the whole step: per stage the algorithmic work over
    the peak of its bound (HBM bytes, or contraction flops on the executed
    triangle), summed over the stages the step runs, against the measured
    step time."""
    per = {}
    for k, v in stages.items():
        _, amount, unit, peak = work[k]
        per[k] = amount / (peak * (1e12 if unit == "TFLOP/s" else 1e9)) * 1e3 * v["calls_per_step"]
    t = sum(per.values())
    return {"t_roof_ms": round(t, 4), "t_measured_ms": round(ms_per_step, 4), "frac": round(t / ms_per_step, 4),
            "stages_roof_ms": {k: round(v, 4) for k, v in per.items()}}


def run_serving(args):
    """Config-5 trace: Poisson arrivals; per request direction 50/50, nside in
    {64,...,1024}, lmax in {2 nside - 1, 3 nside - 1}, 1..32 FP32 channels, inputs
    from per-(nside, lmax) pools synthesised beforehand (not timed).  Served by the
    serving loop (budget, slots) and, as the baseline, one at a time in arrival
    order on one stream."""
    import torch
    import paper_2510_01785_amd as shtx
    from paper_2510_01785_amd.serve import Request, Server
    dev = torch.device("cuda:0")
    rng = np.random.default_rng(17856)
    nsides = [64, 128, 256, 512, 1024]
    n = args.requests
    arrivals = np.cumsum(rng.exponential(1.0 / args.rate, n))
    trace = []
    for i in range(n):
        nside = int(rng.choice(nsides))
        lmax = int(rng.choice([2 * nside - 1, 3 * nside - 1]))
        trace.append(("map2alm" if rng.random() < 0.5 else "alm2map", nside, lmax, int(rng.integers(1, 33))))
    print("[bench] serving: %d requests at %.0f/s; building pools and tables" % (n, args.rate), flush=True)
    pools = {}
    for nside in nsides:
        g = torch.Generator(device=dev).manual_seed(nside)
        pools[("map", nside)] = torch.randn(32, 12 * nside * nside, device=dev, generator=g)
        for lmax in (2 * nside - 1, 3 * nside - 1):
            na = (lmax + 1) * (lmax + 2) // 2
            pools[("alm", lmax)] = torch.randn(32, na, device=dev, dtype=torch.complex64, generator=g)
            shtx.get_tables(nside, lmax, dev)
    torch.cuda.synchronize()

    def data(d, nside, lmax, B):
        return pools[("map", nside)][:B] if d == "map2alm" else pools[("alm", lmax)][:B]

    # warm both paths (kernel loads) on one small request of each kind
    for d, nside, lmax, B in trace[:4]:
        x = data(d, nside, lmax, B)
        shtx.map2alm_raw(x, lmax) if d == "map2alm" else shtx.alm2map_raw(x, nside, lmax)
    torch.cuda.synchronize()
    budget = int(args.budget_gib * (1 << 30))
    srv = Server(dev, budget_bytes=budget, slots=args.slots, max_merge_channels=args.merge_channels)
    print("[bench] serving loop run", flush=True)
    errors = []

    def check(f):  # outputs are dropped as soon as they are done
        if f.exception() is not None:
            errors.append(f.exception())

    t0 = time.perf_counter()
    for (d, nside, lmax, B), ta in zip(trace, arrivals):
        now = time.perf_counter() - t0
        if ta > now:
            time.sleep(ta - now)
        srv.submit(Request(d, nside, lmax, data(d, nside, lmax, B))).add_done_callback(check)
    srv.drain()
    st = srv.stats()
    srv.close()
    torch.cuda.synchronize()
    if errors:
        raise errors[0]
    print("[bench] one-at-a-time run", flush=True)
    lat = []
    t0 = time.perf_counter()
    for (d, nside, lmax, B), ta in zip(trace, arrivals):
        now = time.perf_counter() - t0
        if ta > now:
            time.sleep(ta - now)
        x = data(d, nside, lmax, B)
        out = shtx.map2alm_raw(x, lmax) if d == "map2alm" else shtx.alm2map_raw(x, nside, lmax)
        torch.cuda.synchronize()
        lat.append(time.perf_counter() - t0 - ta)
        del out
    wall1 = time.perf_counter() - t0
    lat = np.array(lat) * 1e3
    maps = sum(t[3] for t in trace)
    out = {
        "metric": "serving: maps/s and p50/p99 request latency on a Poisson trace of mixed transforms",
        "value": round(st["maps_per_s"], 3),
        "unit": "maps/s",
        "n_gpus": 1,
        "higher_is_better": True,
        "dtype": "f32",
        "data": "synthetic",
        "p50_ms": round(st["p50_ms"], 3),
        "p99_ms": round(st["p99_ms"], 3),
        "queue_wait_p99_ms": round(st["queue_wait_p99_ms"], 3),
        "peak_in_use_gib": round(st["peak_in_use_bytes"] / (1 << 30), 3),
        "launches": st["launches"],
        "one_at_a_time": {"maps_per_s": round(maps / wall1, 3), "p50_ms": round(float(np.percentile(lat, 50)), 3),
                          "p99_ms": round(float(np.percentile(lat, 99)), 3)},
        "config": {"workload": "healpix_sht_serving", "requests": n, "rate_per_s": args.rate,
                   "nside": nsides, "lmax": "2N-1 or 3N-1", "channels": "1..32", "direction": "50/50",
                   "budget_gib": args.budget_gib, "slots": args.slots, "merge_channels": args.merge_channels},
    }
    print(json.dumps(out), flush=True)


def run_grad(args):
    """Differentiable workload: forward map2alm of B maps at Nside (default
    1024, lmax 2047, B 16), the spectral loss sum_l w_l sum_m |a_lm|^2 with
    w_l = 1/(l+1), and its backward through the hand-written adjoint chain
    (torch.autograd.Function) to the gradient map; FP32 or BF16 maps.  One
    step = forward + loss + backward; the loss's elementwise terms run as torch
    operations on the coefficients (0.27 GB at the default size)."""
    import torch
    import paper_2510_01785_amd as shtx
    from paper_2510_01785_amd import _lib, synth
    dev = torch.device("cuda:0")
    nside, B = args.nside, args.batch
    lmax = args.lmax if args.lmax is not None else 2 * nside - 1
    dt = {"f32": torch.float32, "f64": torch.float64, "bf16": torch.bfloat16}[args.dtype]
    print("[bench] grad nside=%d lmax=%d B=%d %s" % (nside, lmax, B, args.dtype), flush=True)
    ct = torch.complex128 if args.dtype == "f64" else torch.complex64
    alm0 = torch.tensor(synth.gaussian_alm(17853, B, lmax, "lp10"), dtype=ct, device=dev)
    x = shtx.alm2map_raw(alm0, nside, lmax).to(dt).requires_grad_(True)
    ls, _ = synth.lm_arrays(lmax)
    wl = torch.tensor(1.0 / (ls + 1.0), device=dev, dtype=torch.float64 if args.dtype == "f64" else torch.float32)

    def step():
        x.grad = None
        a = shtx.map2alm(x, lmax)
        loss = (wl * (a.real ** 2 + a.imag ** 2)).sum()
        loss.backward()
        return a

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    L = _lib.lib()
    L.shtx_profile_reset()
    L.shtx_profile_enable(1)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    stream = torch.cuda.current_stream(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        evs[i][0].record(stream)
        step()
        evs[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    L.shtx_profile_enable(0)
    prof = _lib.profile_read()
    lat = np.array([u.elapsed_time(v) for u, v in evs])
    a = step().detach()
    torch.cuda.synchronize()
    out = {
        "metric": "differentiable SHT: forward + spectral loss + adjoint backward, maps/s at Nside=%d lmax=%d B=%d"
                  % (nside, lmax, B),
        "value": round(B * args.steps / wall, 3),
        "unit": "maps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1000.0 * wall / args.steps, 4),
        "p50_ms": round(float(np.percentile(lat, 50)), 4),
        "p99_ms": round(float(np.percentile(lat, 99)), 4),
        "higher_is_better": True,
        "dtype": args.dtype,
        "data": "synthetic",
        "stages_ms_per_step": {k: round(v[0] / args.steps, 4) for k, v in prof.items() if v[1]},
        "config": {"workload": "healpix_sht_grad", "nside": nside, "lmax": lmax, "batch": B,
                   "loss": "sum_l w_l sum_m |a_lm|^2, w_l = 1/(l+1)", "fields": "gaussian C_l=(l+10)^-2"},
    }
    if not args.no_cpu_baseline:
        # the oracle on channel 0: forward of the timed map and the adjoint of
        # the loss gradient of the step's own coefficients
        print("[bench] oracle on channel 0 of the step", flush=True)
        from oracle import _clib, sht
        _clib.build()
        f0 = x.detach()[0].double().cpu().numpy()
        a0 = a[0].cpu().numpy().astype(np.complex128)
        g0 = x.grad[0].double().cpu().numpy()
        t1 = time.perf_counter()
        a_ref = sht.map2alm(f0[None, :], lmax, nside)[0]
        g_ref = sht.map2alm_backward(sht.spectral_loss_grad(a0[None, :], lmax), nside, lmax)[0]
        dt_o = time.perf_counter() - t1
        out["accuracy_vs_oracle"] = {"map2alm_rel_l2": float("%.3e" % rel_l2(a0, a_ref)),
                                     "grad_map_rel_l2": float("%.3e" % rel_l2(g0, g_ref)),
                                     "oracle": "FP64 CPU oracle on channel 0 of the timed step"}
        out["cpu_baseline"] = dict(value=round(1.0 / dt_o, 5), unit="maps/s", cores=_clib.threads(), kind="oracle",
                                   sample="channel 0: oracle forward + adjoint, %.1f s" % dt_o)
    print(json.dumps(out), flush=True)


def run_peaks():
    """Measured counterparts of the published peaks: a 4 GiB device copy
    (HBM read + write) and large GEMMs in FP32, FP64 and BF16 (library
    kernels on the matrix cores), each the best of 5 timed runs."""
    import torch
    dev = torch.device("cuda:0")

    def best(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) / 1000.0)
        return min(ts)
    n = (4 << 30) // 4
    src = torch.ones(n, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    t = best(lambda: dst.copy_(src))
    out = {"hbm_copy_GBs": round(2 * 4 * n / t / 1e9, 1)}
    del src, dst
    for name, dt, k in (("fp32_gemm_TFs", torch.float32, 8192), ("fp64_gemm_TFs", torch.float64, 8192),
                        ("bf16_gemm_TFs", torch.bfloat16, 16384)):
        a = torch.randn(k, k, device=dev).to(dt)
        b = torch.randn(k, k, device=dev).to(dt)
        t = best(lambda: torch.matmul(a, b))
        out[name] = round(2.0 * k ** 3 / t / 1e12, 1)
        del a, b
    out["published"] = {"hbm_GBs": PEAK["hbm_GBs"], "fp32_mfma_TFs": PEAK["fp32_mfma_TFs"],
                        "fp64_mfma_TFs": 78.6, "bf16_mfma_TFs": 2500.0}
    print(json.dumps(out), flush=True)


def run_jacobi(args):
    """3-iteration refined analysis (Eq. (4)) of one map at Nside=2048,
    lmax=4095 (4 forward + 3 inverse transforms), FP64 or FP32; the field is a
    band-limited Gaussian random field with C_l = l^-2."""
    import torch
    import paper_2510_01785_amd as shtx
    from paper_2510_01785_amd import synth
    dev = torch.device("cuda:0")
    nside = args.nside if args.nside != 1024 else 2048  # the refinement workload's default size
    lmax = 2 * nside - 1
    dt = torch.float64 if args.dtype == "f64" else torch.float32
    ct = torch.complex128 if args.dtype == "f64" else torch.complex64
    print("[bench] jacobi nside=%d lmax=%d %s" % (nside, lmax, args.dtype), flush=True)
    a0 = torch.tensor(synth.gaussian_alm(17855, 1, lmax, "l_m2"), dtype=ct, device=dev)
    f = shtx.alm2map_raw(a0, nside, lmax).to(dt)
    from paper_2510_01785_amd import _lib
    for _ in range(args.warmup):
        shtx.map2alm_iter(f, lmax, 3)
    torch.cuda.synchronize()
    L = _lib.lib()
    L.shtx_profile_reset()
    L.shtx_profile_enable(1)
    evs = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        a = shtx.map2alm_iter(f, lmax, 3)
        e1.record()
        evs.append((e0, e1))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    L.shtx_profile_enable(0)
    prof = _lib.profile_read()
    stages = {k: round(v[0] / args.steps, 3) for k, v in prof.items() if v[1]}
    lat = np.array([x.elapsed_time(y) for x, y in evs])
    err = [float((torch.linalg.vector_norm(shtx.map2alm_iter(f, lmax, k) - a0) /
                  torch.linalg.vector_norm(a0)).item()) for k in range(4)]
    # accuracy curve of the quadrature weight schemes (Sec. IV-A): equal
    # weights and least-squares ring weights (host helper), per iteration:
    # error against the input coefficients and round trip f - S(a) (RMS and
    # max, relative to f)
    from paper_2510_01785_amd import quadrature
    print("[bench] jacobi accuracy curve (ring weights for nside %d)" % nside, flush=True)
    w_pair = torch.tensor(quadrature.ring_weights_lsq(nside, lmax), dtype=torch.float64)
    curve = {}
    for name, rw in (("equal", None), ("ring", w_pair)):
        rows = []
        for k in range(5):
            a = shtx.map2alm_iter_weighted(f, lmax, k, ring_weights=rw)
            d = f - shtx.alm2map_raw(a, nside, lmax).to(f.dtype)
            rows.append({"iteration": k,
                         "alm_rel_l2": float("%.3e" % (torch.linalg.vector_norm(a - a0) /
                                                      torch.linalg.vector_norm(a0)).item()),
                         "round_trip_rms_rel": float("%.3e" % (d.pow(2).mean().sqrt() / f.pow(2).mean().sqrt()).item()),
                         "round_trip_max_rel": float("%.3e" % (d.abs().max() / f.abs().max()).item())})
        curve[name] = rows
    out = {
        "metric": "3-iteration refined map2alm, Nside=2048 lmax=4095, one map",
        "value": round(1000.0 * wall / args.steps, 3),
        "unit": "ms",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "p50_ms": round(float(np.percentile(lat, 50)), 3),
        "p99_ms": round(float(np.percentile(lat, 99)), 3),
        "higher_is_better": False,
        "dtype": args.dtype,
        "data": "synthetic",
        "rel_error_vs_input_alm_per_iteration": [float("%.3e" % e) for e in err],
        "accuracy_curve_by_weights": curve,
        "stages_ms_per_step": stages,
        "config": {"workload": "healpix_sht_jacobi", "nside": nside, "lmax": lmax, "batch": 1, "iterations": 3,
                   "fields": "gaussian C_l=l^-2"},
    }
    print(json.dumps(out), flush=True)


def run_reorder(args):
    """RING <-> NESTED conversion of B maps at Nside (default 1024, B=16,
    FP32): HBM-bound permutation, each pixel read and written once."""
    import torch
    import paper_2510_01785_amd as shtx
    dev = torch.device("cuda:0")
    nside, B = args.nside, args.batch
    dt = {"f32": torch.float32, "f64": torch.float64, "bf16": torch.bfloat16}[args.dtype]
    n = 12 * nside * nside
    print("[bench] reorder nside=%d batch=%d %s" % (nside, B, args.dtype), flush=True)
    x = torch.randn((B, n), device=dev, dtype=torch.float32).to(dt)
    res = {}
    for name, fn in (("nest2ring", shtx.nest2ring), ("ring2nest", shtx.ring2nest)):
        for _ in range(args.warmup):
            fn(x)
        torch.cuda.synchronize()
        evs = []
        for _ in range(args.steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn(x)
            e1.record()
            evs.append((e0, e1))
        torch.cuda.synchronize()
        ms = np.array([a.elapsed_time(b) for a, b in evs])
        res[name] = float(np.median(ms))
    nbytes = 2.0 * n * B * x.element_size()  # every pixel read once and written once
    gbs = {k: nbytes / (v * 1e-3) / 1e9 for k, v in res.items()}
    cpu = None
    if not args.no_cpu_baseline:
        from oracle import nested
        m = x[0].float().cpu().numpy()
        t0 = time.perf_counter()
        reps = 0
        while time.perf_counter() - t0 < 10.0:
            nested.nest_to_ring(m, nside)
            reps += 1
        el = time.perf_counter() - t0
        cpu = {"value": round(reps * n * 4 * 2 / el / 1e9, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
               "sample": "nest_to_ring of one channel, %d repetitions in %.1f s" % (reps, el)}
    worst = min(gbs.values())
    out = {
        "metric": "RING<->NESTED map reorder GB/s (read + write), Nside=%d B=%d" % (nside, B),
        "value": round(worst, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_call": {k: round(v, 4) for k, v in res.items()},
        "gb_per_s": {k: round(v, 1) for k, v in gbs.items()},
        "higher_is_better": True,
        "dtype": args.dtype,
        "data": "synthetic",
        "roofline": {"kernel": "k_reorder", "bound": "hbm", "achieved": round(worst, 1), "peak": 8000.0,
                     "unit": "GB/s", "frac": round(worst / 8000.0, 4), "traffic": None},
        "cpu_baseline": cpu,
        "config": {"workload": "healpix_reorder", "nside": nside, "batch": B},
    }
    print(json.dumps(out), flush=True)


def run_nested(args):
    """Analysis of NESTED-ordered maps (default Nside 1024, lmax 2047, B 16,
    FP32): the layout conversion fused into the ring FFT's loads
    (map2alm_nested) against the two passes nest2ring + map2alm, and the ring
    FFT's time with NESTED against RING input (HIP events on the stream)."""
    import torch
    import paper_2510_01785_amd as shtx
    from paper_2510_01785_amd import _lib
    dev = torch.device("cuda:0")
    nside, B = args.nside, args.batch
    lmax = args.lmax if args.lmax is not None else 2 * nside - 1
    dt = {"f32": torch.float32, "f64": torch.float64, "bf16": torch.bfloat16}[args.dtype]
    print("[bench] nested-input analysis nside=%d lmax=%d B=%d %s" % (nside, lmax, B, args.dtype), flush=True)
    xr = torch.randn((B, 12 * nside * nside), device=dev, dtype=torch.float32).to(dt)
    xn = shtx.ring2nest(xr)
    shtx.get_tables(nside, lmax, dev)
    L = _lib.lib()
    res = {}
    for name, fn in (("fused", lambda: shtx.map2alm_nested_raw(xn, lmax)),
                     ("two_pass", lambda: shtx.map2alm_raw(shtx.nest2ring(xn), lmax)),
                     ("ring_input", lambda: shtx.map2alm_raw(xr, lmax))):
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        L.shtx_profile_reset()
        L.shtx_profile_enable(1)
        evs = []
        for _ in range(args.steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            evs.append((e0, e1))
        torch.cuda.synchronize()
        L.shtx_profile_enable(0)
        prof = _lib.profile_read()
        res[name] = {"ms_per_call": round(float(np.median([a.elapsed_time(b) for a, b in evs])), 4),
                     "ring_fft_fwd_ms": round(prof["ring_fft_fwd"][0] / max(prof["ring_fft_fwd"][1], 1), 4)}
    out = {
        "metric": "map2alm of NESTED maps, fused layout conversion vs nest2ring + map2alm, Nside=%d lmax=%d B=%d"
                  % (nside, lmax, B),
        "value": round(B / (res["fused"]["ms_per_call"] * 1e-3), 3),
        "unit": "maps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "higher_is_better": True,
        "dtype": args.dtype,
        "data": "synthetic",
        "calls": res,
        "fft_nested_over_ring": round(res["fused"]["ring_fft_fwd_ms"] / res["ring_input"]["ring_fft_fwd_ms"], 4),
        "config": {"workload": "healpix_map2alm_nested", "nside": nside, "lmax": lmax, "batch": B},
    }
    print(json.dumps(out), flush=True)


def run_resize(args):
    """Spectral resize of B coefficient sets from lmax = 2 nside - 1 to
    4 nside - 1 (default 2047 -> 4095, B=16, FP32): HBM-bound copy with zero
    fill, input read once and output written once."""
    import torch
    import paper_2510_01785_amd as shtx
    from paper_2510_01785_amd import synth
    dev = torch.device("cuda:0")
    lin, lout, B = 2 * args.nside - 1, 4 * args.nside - 1, args.batch
    ct = torch.complex128 if args.dtype == "f64" else torch.complex64
    print("[bench] resize %d -> %d batch=%d %s" % (lin, lout, B, args.dtype), flush=True)
    x = torch.tensor(synth.gaussian_alm(17853, B, lin, "lp10"), dtype=ct).to(dev)
    res = {}
    for name, (a, b, src) in (("extend", (lin, lout, x)), ("truncate", (lout, lin, None))):
        if src is None:
            src = shtx.alm_resize(x, lin, lout)
        for _ in range(args.warmup):
            shtx.alm_resize(src, a, b)
        torch.cuda.synchronize()
        evs = []
        for _ in range(args.steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            shtx.alm_resize(src, a, b)
            e1.record()
            evs.append((e0, e1))
        torch.cuda.synchronize()
        ms = float(np.median([u.elapsed_time(v) for u, v in evs]))
        na, nb = (a + 1) * (a + 2) // 2, (b + 1) * (b + 2) // 2
        nbytes = (min(na, nb) + nb) * B * x.element_size()  # kept coefficients read, output written
        res[name] = (ms, nbytes / (ms * 1e-3) / 1e9)
    worst = min(v[1] for v in res.values())
    out = {
        "metric": "spectral resize GB/s (read + write), lmax %d <-> %d, B=%d" % (lin, lout, B),
        "value": round(worst, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_call": {k: round(v[0], 4) for k, v in res.items()},
        "gb_per_s": {k: round(v[1], 1) for k, v in res.items()},
        "higher_is_better": True,
        "dtype": args.dtype,
        "data": "synthetic",
        "roofline": {"kernel": "k_alm_resize", "bound": "hbm", "achieved": round(worst, 1), "peak": 8000.0,
                     "unit": "GB/s", "frac": round(worst / 8000.0, 4), "traffic": None},
        "config": {"workload": "healpix_alm_resize", "lmax_in": lin, "lmax_out": lout, "batch": B},
    }
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the transform is not sharded across GPUs; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    if args.calibrate_copy_mib:
        n = args.calibrate_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": 4 * n, "copies": 5}))
        return
    if args.peaks:
        return run_peaks()
    if args.workload == "serving":
        return run_serving(args)
    if args.workload == "jacobi":
        return run_jacobi(args)
    if args.workload == "reorder":
        return run_reorder(args)
    if args.workload == "resize":
        return run_resize(args)
    if args.workload == "grad":
        return run_grad(args)
    if args.workload == "nested":
        return run_nested(args)
    import paper_2510_01785_amd as shtx
    from paper_2510_01785_amd import _lib, synth

    nside, B = args.nside, args.batch
    lmax = args.lmax if args.lmax is not None else 2 * nside - 1
    dt = {"f32": torch.float32, "f64": torch.float64, "bf16": torch.bfloat16}[args.dtype]
    ct = torch.complex128 if args.dtype == "f64" else torch.complex64
    dev = torch.device("cuda:0")
    seed = 17853
    print("[bench] setup nside=%d lmax=%d B=%d %s" % (nside, lmax, B, args.dtype), flush=True)
    alm0 = torch.tensor(synth.gaussian_alm(seed, B, lmax, "lp10"), dtype=ct, device=dev)
    shtx.get_tables(nside, lmax, dev)
    executed, full = shtx.tables_work(nside, lmax, dev)
    map_dtype = torch.float64 if args.dtype == "f64" else torch.float32
    maps = shtx.alm2map_raw(alm0.to(torch.complex128 if map_dtype == torch.float64 else torch.complex64),
                            nside, lmax).to(dt)
    torch.cuda.synchronize()
    L = _lib.lib()

    def step():
        a = shtx.map2alm_raw(maps, lmax)
        if args.dtype == "bf16":
            return a
        return shtx.alm2map_raw(a, nside, lmax)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print("[bench] warmup done", flush=True)
    stream = torch.cuda.current_stream(dev)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    L.shtx_profile_reset()
    L.shtx_profile_enable(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        evs[i][0].record(stream)
        step()
        evs[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    L.shtx_profile_enable(0)
    prof = _lib.profile_read()
    lat = np.array([a.elapsed_time(b) for a, b in evs])
    print("[bench] timed %d steps in %.3f s" % (args.steps, wall), flush=True)
    # the step's outputs for channel 0 (the transforms are deterministic: the
    # same values as every timed step), kept for the oracle comparison
    a_step = shtx.map2alm_raw(maps, lmax)
    f0 = maps[0].double().cpu().numpy()
    a0_gpu = a_step[0].cpu().numpy()
    g0_gpu = None if args.dtype == "bf16" else shtx.alm2map_raw(a_step, nside, lmax)[0].double().cpu().numpy()
    del a_step

    value = B * args.steps / wall
    ms_per_step = 1000.0 * wall / args.steps
    stored = None
    if args.dtype == "bf16" and args.stored_lambda:
        # the same forward with lambda read from the resident stored table
        # (built once, outside the timed region) instead of the recurrence
        print("[bench] stored-lambda table build", flush=True)
        lam = shtx.get_lambda_table(nside, lmax, dev)
        torch.cuda.synchronize()
        for _ in range(args.warmup):
            shtx.map2alm_stored_raw(maps, lmax)
        torch.cuda.synchronize()
        L.shtx_profile_reset()
        L.shtx_profile_enable(1)
        t1 = time.perf_counter()
        for _ in range(args.steps):
            shtx.map2alm_stored_raw(maps, lmax)
        torch.cuda.synchronize()
        wall_s = time.perf_counter() - t1
        L.shtx_profile_enable(0)
        ps = _lib.profile_read()
        a_st = shtx.map2alm_stored_raw(maps, lmax)
        same = bool(torch.equal(a_st, shtx.map2alm_raw(maps, lmax)))
        stored = {"maps_per_s": round(B * args.steps / wall_s, 3), "ms_per_call": round(1000.0 * wall_s / args.steps, 4),
                  "legendre_fwd_ms": round(ps["legendre_fwd"][0] / max(ps["legendre_fwd"][1], 1), 4),
                  "table_gb": round(lam.numel() / 1e9, 3),
                  "table_read_gb_per_s": round(lam.numel() / (ps["legendre_fwd"][0] / max(ps["legendre_fwd"][1], 1) * 1e-3)
                                               / 1e9, 1),
                  "bit_identical_to_recurrence": same}
        del lam, a_st
        shtx.release_lambda_tables()
    # roofline of the dominant stage
    stages = {k: dict(ms_per_call=v[0] / max(v[1], 1), calls=v[1], calls_per_step=v[1] / args.steps)
              for k, v in prof.items() if v[1]}
    dom = max(stages, key=lambda k: stages[k]["ms_per_call"])
    csize = 16 if args.dtype == "f64" else 8
    esize = {"f32": 4, "f64": 8, "bf16": 2}[args.dtype]
    npix = 12 * nside * nside
    spec_bytes = 2 * (lmax + 1) * 2 * nside * B * csize
    alm_bytes = (lmax + 1) * (lmax + 2) // 2 * B * csize
    mfma = dom.startswith("legendre") and on_mfma(dom, args.dtype, B)
    # Legendre work: 4 flops (complex += real * complex) per executed (l, m,
    # ring pair) triple and channel; the executed triangle skips the l where
    # lambda_lm(z_p) is negligible (the full triangle is reported beside it)
    bf_ = "mfma" if on_mfma("legendre_fwd", args.dtype, B) else "alu"
    bi_ = "mfma" if on_mfma("legendre_inv", args.dtype, B) else "alu"
    # BF16 spectra: 4 bytes per complex value
    spec_fwd = spec_bytes // 2 if bf16_mfma("legendre_fwd", args.dtype, B) else spec_bytes
    work = {
        # algorithmic work per call of each stage: (bound, amount, unit, peak)
        "legendre_fwd": (bf_, 4.0 * executed * B, "TFLOP/s", stage_peak(bf_, args.dtype) / 1e12),
        "legendre_inv": (bi_, 4.0 * executed * B, "TFLOP/s", stage_peak(bi_, args.dtype) / 1e12),
        "ring_fft_fwd": ("hbm", float(npix * B * esize + spec_fwd), "GB/s", PEAK["hbm_GBs"]),
        "ring_fft_inv": ("hbm", float(npix * B * esize + spec_bytes), "GB/s", PEAK["hbm_GBs"]),
        "alm_in": ("hbm", 2.0 * alm_bytes, "GB/s", PEAK["hbm_GBs"]),
        # BF16 spectra read, operand-order copy written (groups of 16
        # channels, blocks of 8 ring pairs, 512 bytes per (group, m, block))
        "pack_bf16": ("hbm", float(spec_fwd + 2 * ((B + 15) // 16) * (lmax + 1) * ((2 * nside + 7) // 8) * 512),
                      "GB/s", PEAK["hbm_GBs"]),
    }
    if bf16_mfma("legendre_fwd", args.dtype, B):
        # BF16 matrix-core analysis: the BF16 contraction (4 T_exec B flops)
        # takes 4 T_exec B / 2.5 PFLOP/s, below the FP64 recurrence it is fed
        # by (a multiply and a fused multiply-add, 3 flops, per executed
        # triple, shared by the channels) at the FP64 vector peak: that binds
        t_mfma = 4.0 * executed * B / (PEAK["bf16_mfma_TFs"] * 1e12)
        t_rec = 3.0 * executed / (PEAK["fp64_vector_TFs"] * 1e12)
        work["legendre_fwd"] = (("alu", 3.0 * executed, "TFLOP/s", PEAK["fp64_vector_TFs"]) if t_rec >= t_mfma else
                                ("mfma", 4.0 * executed * B, "TFLOP/s", PEAK["bf16_mfma_TFs"]))
    bound, amount, unit, peak = work[dom]
    sec = stages[dom]["ms_per_call"] / 1000.0
    achieved = amount / sec / (1e12 if unit == "TFLOP/s" else 1e9)
    workload = "nside%d_lmax%d_b%d_%s" % (nside, lmax, B, args.dtype)
    kname, kfile = stage_kernel(dom, args.dtype, B)
    traffic = measured_traffic(kname, kfile, workload) if (mfma or unit != "TFLOP/s" or
                                                          bf16_mfma(dom, args.dtype, B)) else None
    roof = dict(kernel=kname, bound=bound, achieved=round(achieved, 3), peak=peak, unit=unit,
                frac=round(achieved / peak, 4), traffic=traffic,
                algorithmic=amount, per="launch" if B <= 16 else "call")
    if unit == "TFLOP/s":
        roof["triples_executed"] = executed
        roof["triples_full"] = full
        roof["achieved_full_triangle"] = round(4.0 * full * B / sec / 1e12, 3)
    out = {
        "metric": ("SHT fwd+inv maps/s at Nside=%d lmax=%d B=%d; %% roofline; p50/p99 latency" % (nside, lmax, B)
                   if args.dtype != "bf16" else
                   "SHT fwd maps/s at Nside=%d lmax=%d B=%d, BF16 maps; %% roofline; p50/p99 latency" % (nside, lmax, B)),
        "value": round(value, 3),
        "unit": "maps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "p50_ms": round(float(np.percentile(lat, 50)), 4),
        "p99_ms": round(float(np.percentile(lat, 99)), 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": "healpix_sht_fwd_inv", "nside": nside, "lmax": lmax, "batch": B,
                   "fields": "gaussian C_l=(l+10)^-2"},
        "stages_ms_per_call": {k: round(v["ms_per_call"], 4) for k, v in stages.items()},
        "roofline": roof,
        "step_roofline": step_roofline(stages, work, args.dtype, B, ms_per_step),
    }
    if stored is not None:
        out["stored_lambda"] = stored
    if not args.no_cpu_baseline:
        print("[bench] oracle on channel 0 of the timed step (accuracy + cpu baseline)", flush=True)
        out["accuracy_vs_oracle"], out["cpu_baseline"] = oracle_check(nside, lmax, f0, a0_gpu, g0_gpu)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
