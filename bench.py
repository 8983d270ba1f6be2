#!/usr/bin/env python3
"""Benchmark: gate-layers/s of the DMRG compression step at chi = 1024 on one GPU.

Workload: 54 qubits on a 6x9 grid read in snake order along its width 6,
random one-qubit gates from {sqrt(X), sqrt(Y), sqrt(W)} and fSim(theta, phi)
two-qubit gates (theta ~ U(0, pi/2), phi ~ U(0, pi)) on the coupler patterns
ABCDCDAB, depth 20, seed 0 (synthetic, generated in-process).  One step is one
``apply_layer_dmrg`` call (zip-up + n_sweeps two-site sweeps of one layer).
The first ``--warmup`` layers bring the bond dimension to chi and are not
timed; the next ``--steps`` layers are timed between two device
synchronisations.  All inputs are resident on the GPU when timing starts (the
gate list of a layer is a few KiB and is copied inside the call).

Prints one JSON line.  ``roofline`` describes the complex-GEMM contraction
kernels: algorithmic flops (8 per complex multiply-add) over the summed launch
durations measured with HIP events on the stream each launch runs on.
``roofline_tridiag`` does the same for the persistent tridiagonal reduction of
the FP64 eigensolver ((16/3) n^3 flops per order-n matrix), the kernel with the
largest total time; it is latency-bound, so it is reported against the FP64
vector peak.  ``sampling`` times bitstring sampling from the final MPS.
``cpu_baseline`` times the FP64 oracle on a bounded sample (see
``cpu_baseline()``).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# dense MFMA TFLOP/s on MI355X; the split path executes six BF16 products per
# algorithmic real product, so its algorithmic peak is 2500 / 6
PEAK = {"fp32": 157.3, "fp64": 78.6, "bf16x3": 2500.0 / 6.0}
DTYPE = {"fp32": "f32", "fp64": "f64", "bf16x3": "bf16x3-f32acc"}
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_cgemm_54q_chi1024.json")
SV_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_sv_2q_32q.json")


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=4)
    p.add_argument("--warmup", type=int, default=4)
    p.add_argument("--chi", type=int, default=1024)
    p.add_argument("--sweeps", type=int, default=2)
    p.add_argument("--precision", choices=("fp32", "bf16x3", "fp64"), default="bf16x3")
    p.add_argument("--seed", type=int, default=0)
    p.add_argument("--compare-fp64", type=int, default=1,
                   help="also time the same layers with FP64 contractions (1 = yes)")
    p.add_argument("--cpu-baseline", type=int, default=1)
    p.add_argument("--single-site", type=int, default=1,
                   help="also time the single-site update (split and FP64) on the same layers (1 = yes)")
    p.add_argument("--samples", type=int, default=65536,
                   help="bitstrings sampled from the final MPS of the timed run (0 = skip)")
    p.add_argument("--multilayer-chi", type=int, default=256,
                   help="chi of the K = 2 layers-per-step leg on the same layers (0 = skip)")
    p.add_argument("--closed-amplitudes", type=int, default=4,
                   help="closed-mode amplitudes timed on the 54-qubit circuit at chi = 64 (0 = skip)")
    p.add_argument("--statevector", type=int, default=32,
                   help="qubits of the exact-statevector leg (a Sycamore-layout circuit; 0 = skip)")
    p.add_argument("--progress", action="store_true", help="print one line per layer to stderr")
    p.add_argument("--calibrate-copy-mib", type=int, default=0,
                   help="fill, then sum, a device buffer of this many MiB (HBM counter calibration)")
    return p.parse_args()


def source_hash() -> str:
    h = hashlib.sha256()
    for name in ("cgemm.hip", "cgemm_bf16.hip"):
        with open(os.path.join(ROOT, "paper_2207_05612_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def mark(torch):
    """A short spin kernel on the current stream: delimits the timed region in profiler traces."""
    torch.cuda._sleep(1000)


def run_layers(mps, circuit, precision, chi, sweeps, warmup, steps, torch, progress=False, samples=0,
               update="two-site"):
    st = mps.MPS(circuit.n, None, max_chi=chi, precision=precision)
    for d in range(warmup):
        f = st.apply_layer_dmrg(circuit.layers[d], chi, sweeps, update=update)
        if progress:
            print("warmup layer %d f=%.6f" % (d, f), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    st.set_profiling(True)
    fs = []
    mark(torch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for d in range(warmup, warmup + steps):
        fs.append(st.apply_layer_dmrg(circuit.layers[d], chi, sweeps, update=update))
        if progress:
            print("timed layer %d f=%.6f" % (d, fs[-1]), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    mark(torch)
    stats = {k: st.kernel_stats(k) for k in ("contract", "mpo", "gram", "tridiag", "eigh", "other")}
    bonds = st.bond_dims()
    fid = st.fidelity()
    sampling = None
    if samples > 0:
        st.sample(min(samples, 4096), seed=1)           # warm-up (buffers, kernels)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st.sample(samples, seed=2)
        torch.cuda.synchronize()
        ts = time.perf_counter() - t0
        # per sample and site: (1 x D_k) (D_k x 2 D_k+1) complex MACs
        flops = 16.0 * samples * sum(bonds[k] * bonds[k + 1] for k in range(len(bonds) - 1))
        sampling = {"samples": samples, "seconds": ts, "samples_per_s": samples / ts,
                    "algorithmic_tflops": flops / ts / 1e12, "max_bond": max(bonds)}
        if progress:
            print("sampled %d bitstrings in %.2f s" % (samples, ts), file=sys.stderr, flush=True)
    st.close()
    return dt, fs, stats, bonds, fid, sampling


def cpu_baseline(chi: int, sweeps: int, stats_per_layer_flops: float, n_steps_per_layer: int,
                 min_seconds: float = 10.0, max_updates: int = 8):
    """Time the FP64 oracle on a bounded sample of the chi = 1024 workload.

    Sample: two-site updates of the oracle (local tensor, truncated SVD and
    environment update) at the workload's chi = 1024 with MPO bonds w = 4
    (an A/B-layer cut), on fresh random inputs of those shapes each time,
    repeated until min_seconds of CPU work have run (at most max_updates).
    The time per layer is extrapolated as (steps per layer) x (mean SVD time)
    + (contraction flops of the GPU's measured layers) / (oracle contraction
    rate), and reported in gate-layers/s.
    """
    import numpy as np
    from oracle import dmrg
    rng = np.random.default_rng(0)

    def rc(*shape):
        return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(np.prod(shape[1:]))

    w = 4
    flops_contract = 8.0 * (chi * 1 * chi * 2 * chi + chi * 2 * w * chi * 2 * chi + 4 * chi * w * chi * chi
                            + chi * 2 * chi * w * chi) + 8.0 * 4 * chi * chi * w * w
    t_con = t_svd = 0.0
    updates = 0
    while updates < max_updates and (updates == 0 or t_con + t_svd < min_seconds):
        lenv, renv = rc(chi, 1, chi), rc(chi, w, chi)
        a1, a2 = rc(chi, 2, chi), rc(chi, 2, chi)
        w1, w2 = rc(1, 2, 2, w), rc(w, 2, 2, w)
        t0 = time.perf_counter()
        th = dmrg.two_site_tensor(lenv, a1, w1, a2, w2, renv)
        t1 = time.perf_counter()
        u, s, vh, total = dmrg.truncated_svd(th.reshape(2 * chi, 2 * chi), chi)
        t2 = time.perf_counter()
        b = u.reshape(chi, 2, -1)
        dmrg.env_left_step(lenv, a1, w1, b)
        t3 = time.perf_counter()
        t_con += (t1 - t0) + (t3 - t2)
        t_svd += t2 - t1
        updates += 1
    rate = flops_contract * updates / t_con
    t_layer = n_steps_per_layer * t_svd / updates + stats_per_layer_flops / rate
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    threads = int(os.environ.get("OMP_NUM_THREADS", cores))
    return {"value": 1.0 / t_layer, "unit": "gate-layers/s", "cores": min(cores, threads), "kind": "oracle",
            "sample": "%d oracle two-site updates (local tensor + zgesdd truncation + environment update) at "
                      "chi=%d, MPO bond 4, fresh random inputs each: %.1f s in total (SVD %.2f s per update, "
                      "contraction %.1f GFLOP/s); per-layer time extrapolated from %d updates per layer and the "
                      "GPU run's algorithmic contraction flops per layer"
                      % (updates, chi, t_con + t_svd, t_svd / updates, rate / 1e9, n_steps_per_layer)}


def multilayer_leg(mps, circuit, precision, chi, sweeps, warmup, steps, torch):
    """The timed layers applied two per compression step (one MPO over both layers) against the
    same layers one per step, both from the same warmed-up state, at a chi where K = 2 fits."""
    out = {"chi": chi, "layers": steps}
    for K in (1, 2):
        st = mps.MPS(circuit.n, None, max_chi=chi, precision=precision)
        for d in range(warmup):
            st.apply_layer_dmrg(circuit.layers[d], chi, sweeps)
        torch.cuda.synchronize()
        st.set_profiling(True)
        t0 = time.perf_counter()
        fs = [st.apply_layers_dmrg(circuit.layers[d:d + K], chi, sweeps)
              for d in range(warmup, warmup + steps, K)]
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        con = st.kernel_stats("contract")
        out["K%d" % K] = {"gate_layers_per_s": steps / dt, "f_steps": fs, "F_tilde": st.fidelity()["F_tilde"],
                          "contraction_tflops": con["flops"] / (con["ms"] * 1e-3) / 1e12 if con["ms"] > 0 else 0.0}
        st.close()
    return out


def closed_leg(circuits, torch, n_amp):
    """Closed-mode amplitudes <x|U|0> of the 54-qubit circuit at chi = 64 (cut after layer 10,
    forward MPS built once, one backward MPS per bitstring), split precision."""
    import numpy as np
    from paper_2207_05612_amd import closed, mps
    c = circuits.sycamore_like_54_workload(0, depth=20)
    t0 = time.perf_counter()
    amps = closed.ClosedAmplitudes(c, chi=64, n_sweeps=1, d1=10, precision=mps.MPS_BF16X3)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    bits = np.random.default_rng(5).integers(0, 2, size=(n_amp, c.n)).astype(np.uint8)
    t0 = time.perf_counter()
    vals = [amps(b) for b in bits]
    torch.cuda.synchronize()
    t_amp = time.perf_counter() - t0
    f_fwd = amps.fwd.fidelity()["F_tilde"]
    amps.close()
    return {"chi": 64, "d1": 10, "amplitudes": n_amp, "forward_s": t_fwd, "amplitudes_per_s": n_amp / t_amp,
            "F_tilde_forward": f_fwd, "F_tilde_backward": [float(np.exp(x)) for x in amps.log_f_backward],
            "abs_amplitudes": [abs(v) for v in vals]}


def statevector_leg(mps, circuits, torch, n_qubits):
    """Gate passes of the exact statevector (HBM-bound: every pass reads and writes all 2^n
    FP64 complex amplitudes) on a Sycamore-layout circuit of n_qubits, timed with HIP events
    on the stream the kernels run on."""
    nb = {28: 4, 32: 5, 33: 6}.get(n_qubits)
    nc = {28: 8, 32: 7, 33: 6}.get(n_qubits)
    if nb is None:
        raise SystemExit("--statevector takes 28, 32 or 33")
    c = circuits.sycamore_circuit(circuits.SycamoreLayout(nb, nc), 8, seed=0, sequence="I")
    g = mps.Statevector(c.n)
    g.apply_layer(c.layers[0])                      # warm-up
    passes = 0
    for layer in c.layers[1:]:
        two = [q for g2 in layer if g2[1] >= 0 for q in (g2[0], g2[1])]
        lone = len({g1[0] for g1 in layer if g1[1] < 0} - set(two))
        passes += len(two) // 2 + (lone + 1) // 2
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for layer in c.layers[1:]:
        g.apply_layer(layer)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    g.close()
    bytes_per_pass = 2.0 * 16.0 * 2.0 ** c.n
    achieved = bytes_per_pass * passes / (ms * 1e-3) / 1e9
    traffic = None
    if os.path.exists(SV_TRAFFIC_FILE):
        # HBM bytes per pass from the FETCH_SIZE / WRITE_SIZE passes; valid for the same kernel source
        rec = json.load(open(SV_TRAFFIC_FILE))
        with open(os.path.join(ROOT, "paper_2207_05612_amd", "csrc", "statevector.hip"), "rb") as fh:
            if rec.get("source_hash") == hashlib.sha256(fh.read()).hexdigest()[:16] and rec.get("n_qubits") == c.n:
                traffic = rec.get("bytes_per_launch")
    return {"n_qubits": c.n, "layers": len(c.layers) - 1, "gate_passes": passes, "ms": ms,
            "ms_per_pass": ms / passes,
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                         "algorithmic_bytes_per_launch": bytes_per_pass,
                         "kernel": "sv_2q_kernel, sv_2q_bit0_kernel (one two-qubit pass over all amplitudes, FP64 planar)"}}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU: the compression step has no multi-GPU path in this build "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    from paper_2207_05612_amd import circuits, mps
    if not os.path.exists(mps.LIB_PATH):
        from paper_2207_05612_amd import build as _b
        _b.build()
    mps.load_library()

    if args.calibrate_copy_mib:
        # known HBM traffic for the counter calibration: a fill writes the buffer once,
        # a sum reads it once
        n = args.calibrate_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        total = src.sum()
        torch.cuda.synchronize()
        del src, total

    c = circuits.sycamore_like_54_workload(args.seed, depth=20)
    if args.warmup + args.steps > len(c.layers):
        raise SystemExit("warmup + steps must not exceed the circuit depth (20)")
    prec = {"fp32": mps.MPS_FP32, "bf16x3": mps.MPS_BF16X3, "fp64": mps.MPS_FP64}[args.precision]
    dt, fs, stats, bonds, fid, sampling = run_layers(mps, c, prec, args.chi, args.sweeps, args.warmup, args.steps,
                                                     torch, args.progress, args.samples)
    value = args.steps / dt
    con = stats["contract"]
    achieved = con["flops"] / (con["ms"] * 1e-3) / 1e12 if con["ms"] > 0 else 0.0
    peak = PEAK[args.precision]
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        # HBM bytes per launch of the same kernel over the same timed launches, from the
        # FETCH_SIZE / WRITE_SIZE passes; only valid for unchanged kernel sources and launch schedule
        rec = json.load(open(TRAFFIC_FILE))
        if (rec.get("source_hash") == source_hash() and rec.get("precision") == args.precision
                and rec.get("timed_region_dispatches") == con["launches"]):
            traffic = rec.get("bytes_per_launch")
    total_flops = sum(v["flops"] for v in stats.values())

    out = {
        "metric": "gate-layers/s & TFLOP/s at chi=1024, split-FP32 vs FP64 on 1 GPU, equal fidelity",
        "value": value,
        "unit": "gate-layers/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {"workload": "54-qubit 6x9 snake, fSim + random 1q gates, depth 20, seed %d; layers %d..%d timed"
                               % (args.seed, args.warmup, args.warmup + args.steps - 1),
                   "chi": args.chi, "n_sweeps": args.sweeps, "contraction_precision": args.precision,
                   "truncation_precision": "fp64", "max_bond": max(bonds)},
        "contraction_tflops": achieved,
        "all_kernels_algorithmic_tflops": total_flops / dt / 1e12,
        "time_split_ms": {k: round(v["ms"], 1) for k, v in stats.items()},
        "class_algorithmic_tflops": {k: round(v["flops"] / (v["ms"] * 1e-3) / 1e12, 2)
                                     for k, v in stats.items() if v["ms"] > 0 and v["flops"] > 0},
        "f_delta": fs,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak, "traffic": traffic,
                     "algorithmic_bytes_per_launch": con["bytes"] / max(con["launches"], 1),
                     "kernel": "%s (complex planar GEMM, %d launches, %.1f ms)"
                               % ("cgemm_bf16x3_nt_kernel" if args.precision == "bf16x3" else
                                  "cgemm_kernel<%s>" % args.precision, con["launches"], con["ms"])},
        "contraction_frac_of_fp32_mfma_peak": achieved / PEAK["fp32"],
    }
    tri = stats["tridiag"]
    if tri["ms"] > 0:
        tri_tf = tri["flops"] / (tri["ms"] * 1e-3) / 1e12
        out["roofline_tridiag"] = {"bound": "alu", "achieved": tri_tf, "peak": PEAK["fp64"], "unit": "TFLOP/s",
                                   "frac": tri_tf / PEAK["fp64"], "traffic": None,
                                   "kernel": "hetrd_kernel (persistent tridiagonal reduction, %d launches, "
                                             "%.1f ms; latency-bound: one cross-workgroup wait per column)"
                                             % (tri["launches"], tri["ms"])}
    if sampling:
        out["sampling"] = sampling
    if args.compare_fp64 and args.precision != "fp64":
        dt64, fs64, stats64, _, _, _ = run_layers(mps, c, mps.MPS_FP64, args.chi, args.sweeps, args.warmup,
                                                  args.steps, torch, args.progress)
        c64 = stats64["contract"]
        out["fp64_path"] = {"value": args.steps / dt64, "unit": "gate-layers/s",
                            "contraction_tflops": c64["flops"] / (c64["ms"] * 1e-3) / 1e12,
                            "time_split_ms": {k: round(v["ms"], 1) for k, v in stats64.items()},
                            "f_delta": fs64}
        out["speedup_vs_fp64"] = value / (args.steps / dt64)
        out["max_rel_f_delta_diff_vs_fp64"] = max(abs(a - b) / b for a, b in zip(fs, fs64))
    if args.single_site:
        ss = {}
        for name, pr in (("split", prec), ("fp64", mps.MPS_FP64)):
            d_ss, f_ss, st_ss, _, _, _ = run_layers(mps, c, pr, args.chi, args.sweeps, args.warmup, args.steps, torch,
                                                    args.progress, 0, update="single-site")
            cs = st_ss["contract"]
            ss[name] = {"value": args.steps / d_ss, "f_delta": f_ss,
                        "contraction_tflops": cs["flops"] / (cs["ms"] * 1e-3) / 1e12 if cs["ms"] > 0 else 0.0,
                        "time_split_ms": {k: round(v["ms"], 1) for k, v in st_ss.items()}}
        out["single_site"] = {"update": "single-site sweeps after the same zip-up (paper's update rule)",
                              "value": ss["split"]["value"], "unit": "gate-layers/s",
                              "speedup_vs_fp64_single_site": ss["split"]["value"] / ss["fp64"]["value"],
                              "split": ss["split"], "fp64": ss["fp64"]}
    if args.multilayer_chi:
        out["multilayer"] = multilayer_leg(mps, c, prec, args.multilayer_chi, args.sweeps, args.warmup, args.steps,
                                           torch)
    if args.closed_amplitudes:
        out["closed"] = closed_leg(circuits, torch, args.closed_amplitudes)
    if args.statevector:
        out["statevector"] = statevector_leg(mps, circuits, torch, args.statevector)
    if args.cpu_baseline:
        layer_flops = con["flops"] / args.steps
        out["cpu_baseline"] = cpu_baseline(args.chi, args.sweeps, layer_flops, (c.n - 1) * (1 + args.sweeps))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
