#!/usr/bin/env python3
"""Benchmark: gate-layers/s of the DMRG compression step at chi = 1024 on one GPU.

Workload: 54 qubits on a 6x9 grid read in snake order along its width 6,
random one-qubit gates from {sqrt(X), sqrt(Y), sqrt(W)} and fSim(theta, phi)
two-qubit gates (theta ~ U(0, pi/2), phi ~ U(0, pi)) on the coupler patterns
ABCDCDAB, depth 20, seed 0 (synthetic, generated in-process).  One step is one
``apply_layer_dmrg`` call (zip-up + n_sweeps two-site sweeps of one layer).
The first ``--warmup`` layers bring the bond dimension to chi and are not
timed; the following layers are timed, at most ``--steps`` of them and never
past the circuit's depth 20 (``steps`` in the output line is the number
actually timed).  All inputs are resident on the GPU when timing starts (the
gate list of a layer is a few KiB and is copied inside the call).

Prints one JSON line.  ``roofline_contraction`` describes the contraction GEMM
kernel: algorithmic flops (8 per complex multiply-add) over the summed launch
durations measured with HIP events on the stream each launch runs on.
``roofline_truncation`` does the same for the persistent FP64 tridiagonal
reduction of the truncation ((16/3) n^3 flops per order-n matrix).
``roofline`` repeats whichever of the two took more time in the timed layers
(the dominant kernel).  Each carries ``traffic``: the HBM bytes per launch from
the FETCH_SIZE / WRITE_SIZE record of the same kernel source under profiles/,
scaled to this run's algorithmic bytes per launch (null when the kernel
changed since).
``fp64_path`` times the all-FP64 path on the first ``--fp64-steps`` of the
same layers; ``speedup_vs_fp64`` compares the two on exactly those layers.
``cpu_baseline`` times the FP64 oracle on a bounded sample (see
``cpu_baseline()``).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

DEPTH = 20
# dense peaks on MI355X (TFLOP/s); a split precision executes several BF16
# products per algorithmic real product, so its algorithmic peak is 2500 / products
PEAK = {"fp32": 157.3, "fp64": 78.6, "bf16x3": 2500.0 / 6.0, "bf16x2": 2500.0 / 3.0}
DTYPE = {"fp32": "f32", "fp64": "f64", "bf16x3": "bf16x3-f32acc", "bf16x2": "bf16x2-f32acc"}
GEMM_KERNEL = {"fp32": "cgemm_kernel<float>", "fp64": "cgemm_kernel<double>",
               "bf16x3": "cgemm_bf16x3_planes_kernel", "bf16x2": "cgemm_bf16x2_planes_kernel"}
GEMM_SOURCE = {"fp32": ("cgemm.hip",), "fp64": ("cgemm.hip",), "bf16x3": ("cgemm_bf16.hip",),
               "bf16x2": ("cgemm_bf16.hip",)}
HBM_PEAK_GBS = 8000.0
PROFILES = os.path.join(ROOT, "profiles")
SV_TRAFFIC_FILE = os.path.join(PROFILES, "traffic_sv_2q_32q.json")
CLASSES = ("contract", "mpo", "gram", "tridiag", "eigh", "other")


def parse(argv=None):
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=15, help="layers timed (at most %d - warmup)" % DEPTH)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--chi", type=int, default=1024)
    p.add_argument("--sweeps", type=int, default=2)
    p.add_argument("--precision", choices=("fp32", "bf16x3", "bf16x2", "fp64"), default="bf16x3")
    p.add_argument("--seed", type=int, default=0)
    p.add_argument("--fp64-steps", type=int, default=8,
                   help="timed layers also run with FP64 contractions (from the first timed layer; 0 = skip)")
    p.add_argument("--cpu-baseline", type=int, default=1)
    p.add_argument("--samples", type=int, default=1000000,
                   help="bitstrings sampled from the final MPS of the timed run, timed, then scored by "
                        "linear XEB against the same MPS's probabilities (0 = skip)")
    p.add_argument("--xeb-fp64", type=int, default=0,
                   help="also build the all-FP64 MPS over the same layers and score the samples with its "
                        "probabilities (1 = yes; about 20 more layer applications)")
    p.add_argument("--single-site", type=int, default=0,
                   help="also time the single-site update (split and FP64) on the same layers (1 = yes)")
    p.add_argument("--multilayer-chi", type=int, default=0,
                   help="chi of a K = 2 layers-per-step leg on the first timed layers (0 = skip)")
    p.add_argument("--closed-amplitudes", type=int, default=0,
                   help="closed-mode amplitudes timed on the 54-qubit circuit at chi = 64 (0 = skip)")
    p.add_argument("--statevector", type=int, default=0,
                   help="qubits of an exact-statevector leg (28, 32 or 33; 0 = skip)")
    p.add_argument("--batched", type=int, default=0,
                   help="instances of the 64-instance ragged batch (n 20..40, depth 8..20, chi 32..512) run "
                        "through apply_layer_dmrg_batched, split precision (0 = skip)")
    p.add_argument("--progress", action="store_true", help="print one line per layer to stderr")
    p.add_argument("--calibrate-copy-mib", type=int, default=0,
                   help="fill, then sum, a device buffer of this many MiB (HBM counter calibration)")
    return p.parse_args(argv)


def source_hash(names) -> str:
    h = hashlib.sha256()
    for name in names:
        with open(os.path.join(ROOT, "paper_2207_05612_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_ratio(kernel: str, sources) -> float | None:
    """Measured HBM bytes per algorithmic byte of `kernel`, from its FETCH_SIZE / WRITE_SIZE
    record under profiles/, if that record was taken on the current kernel source."""
    path = os.path.join(PROFILES, "traffic_%s.json" % kernel.replace("<", "_").replace(">", ""))
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_hash") != source_hash(sources):
        return None
    return rec.get("bytes_per_algorithmic_byte")


def mark(torch):
    """A short spin kernel on the current stream: delimits the timed region in profiler traces."""
    torch.cuda._sleep(1000)


def log(progress, msg):
    if progress:
        print(msg, file=sys.stderr, flush=True)


def run_layers(mps, circuit, precision, chi, sweeps, warmup, steps, torch, progress=False, samples=0,
               update="two-site", tag="", keep=False):
    """Warm up on layers [0, warmup), then time layers [warmup, warmup + steps) one call each.
    Returns per-layer seconds, f_delta, per-layer kernel statistics and the final state's data
    (and the state itself when keep is set; the caller closes it)."""
    st = mps.MPS(circuit.n, None, max_chi=chi, precision=precision)
    for d in range(warmup):
        f = st.apply_layer_dmrg(circuit.layers[d], chi, sweeps, update=update)
        log(progress, "%swarmup layer %d f=%.6f" % (tag, d, f))
    torch.cuda.synchronize()
    st.set_profiling(True)
    secs, fs, per_layer, bonds_per_layer = [], [], [], []
    prev = {k: st.kernel_stats(k) for k in CLASSES}
    mark(torch)
    torch.cuda.synchronize()
    for d in range(warmup, warmup + steps):
        t0 = time.perf_counter()
        fs.append(st.apply_layer_dmrg(circuit.layers[d], chi, sweeps, update=update))
        torch.cuda.synchronize()
        secs.append(time.perf_counter() - t0)
        cur = {k: st.kernel_stats(k) for k in CLASSES}
        per_layer.append({k: {f: cur[k][f] - prev[k][f] for f in cur[k]} for k in CLASSES})
        bonds_per_layer.append(st.bond_dims())
        prev = cur
        log(progress, "%stimed layer %d f=%.6f %.2f s" % (tag, d, fs[-1], secs[-1]))
    mark(torch)
    torch.cuda.synchronize()
    stats = {k: st.kernel_stats(k) for k in CLASSES}
    bonds = st.bond_dims()
    fid = st.fidelity()
    counters = st.counters()
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
        log(progress, "%ssampled %d bitstrings in %.2f s" % (tag, samples, ts))
    out = {"secs": secs, "f": fs, "per_layer": per_layer, "stats": stats, "bonds": bonds, "fid": fid,
           "sampling": sampling, "counters": counters, "bonds_per_layer": bonds_per_layer}
    if keep:
        out["state"] = st
    else:
        st.close()
    return out


def xeb_leg(analysis, sampler, reference, n_samples, torch, label):
    """eq:FB-estim over n_samples bitstrings drawn from `sampler`, scored with the
    probabilities of `reference` (FP64 amplitude evaluation in the library)."""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    est, sd, _ = analysis.linear_xeb(sampler, reference, n_samples, seed=12345)
    torch.cuda.synchronize()
    return {"samples": n_samples, "F_B": est, "F_B_standard_error": sd, "reference": label,
            "seconds": time.perf_counter() - t0}


def tflops(stat):
    return stat["flops"] / (stat["ms"] * 1e-3) / 1e12 if stat["ms"] > 0 else 0.0


# ------------------------------------------------------------- CPU baseline
def _oracle_step_flops(chi, wl, wm, wr):
    """Complex MACs x 8 of one oracle two-site step at bond chi (every bond chi, MPO
    bonds wl, wm, wr) -- the einsum contractions of two_site_tensor and env_left_step,
    with the dense MPO tensors the oracle uses -- and of its SVD of the 2chi x 2chi
    local tensor (~ 22 m^3 for a square complex zgesdd with vectors; a flop-count model
    used only to scale a timed sample to chi = 1024)."""
    c = chi
    macs = (c * wl * c * 2 * c                 # L A
            + c * wl * 2 * c * 2 * wm          # . W (dense)
            + c * 2 * wm * c * 2 * c           # . A
            + c * 2 * wm * 2 * c * 2 * 2 * wr  # . W (dense)
            + c * 4 * wr * c * c               # . R
            + c * wl * c * 2 * c + c * wl * 2 * c * 2 * wm + c * 2 * wm * c * c)   # environment
    return 8.0 * macs, 22.0 * 8.0 * (2 * c) ** 3


def _oracle_zip_flops(chi, wl, wm):
    """The oracle's zip-up step: T = C A W (C of shape chi x wl x chi), then the SVD of the
    2chi x (wm chi) matrix T (~ 4 m^2 n + 22 m^3 complex, m = 2chi <= n)."""
    c = chi
    macs = c * wl * c * 2 * c + c * wl * 2 * c * 2 * wm
    m, n = 2 * c, wm * c
    return 8.0 * macs, 8.0 * (4.0 * m * m * n + 22.0 * m ** 3)


def _time_oracle_step(chi, wl, wm, wr, rng):
    """One oracle two-site step (local tensor, truncated SVD, environment update) and one
    oracle zip-up step on random inputs of the given shapes: seconds (contract, svd) each."""
    import numpy as np
    from oracle import dmrg

    def rc(*shape):
        return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(np.prod(shape[1:]))

    lenv, renv = rc(chi, wl, chi), rc(chi, wr, chi)
    a1, a2 = rc(chi, 2, chi), rc(chi, 2, chi)
    w1, w2 = rc(wl, 2, 2, wm), rc(wm, 2, 2, wr)
    t0 = time.perf_counter()
    th = dmrg.two_site_tensor(lenv, a1, w1, a2, w2, renv)
    t1 = time.perf_counter()
    u, s, vh, _ = dmrg.truncated_svd(th.reshape(2 * chi, 2 * chi), chi)
    t2 = time.perf_counter()
    dmrg.env_left_step(lenv, a1, w1, u.reshape(chi, 2, -1))
    t3 = time.perf_counter()
    step = (t1 - t0 + t3 - t2, t2 - t1)
    del th, u, s, vh
    t0 = time.perf_counter()
    t = np.einsum("pba,atx,bstc->pscx", lenv, a1, w1, optimize=True)
    t1 = time.perf_counter()
    dmrg.truncated_svd(t.reshape(2 * chi, wm * chi), chi)
    t2 = time.perf_counter()
    return step, (t1 - t0, t2 - t1)


def _sample_chi(chi, w, budget):
    """Largest power-of-two bond <= chi whose oracle step and zip-up step stay within
    `budget` operations in total (the sample's size)."""
    c = chi
    while c > 16:
        if sum(_oracle_step_flops(c, w, w, w)) + sum(_oracle_zip_flops(c, w, w)) <= budget:
            break
        c //= 2
    return c


def cpu_baseline(chi, n_sites, sweeps, layer_classes, bonds_per_layer, budgets=(6e12, 2.5e11)):
    """The FP64 oracle on a bounded sample of the timed layers.

    For each layer class of the timed layers (A/B: MPO bonds <= 4; C: <= 256; D: <= 64,
    the class's largest MPO bond in the middle of the step), one oracle two-site step and
    one oracle zip-up step run on random inputs at the class's MPO bond and the largest
    power-of-two bond dimension <= chi whose operation count fits the sample budget
    (budgets[0] with all cores, budgets[1] with one thread).  Each timed part is scaled
    to chi by the ratio of the oracle's own operation counts at the two sizes (1 when the
    sample ran at chi), and a layer costs (n - 1) zip-up steps + sweeps (n - 1) two-site
    steps weighted by sum_k (chi_k/chi)^3 over its cuts (the bond profile the GPU run
    reached).  Reported: timed layers over the summed layer times, all cores and one
    thread."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    rng = np.random.default_rng(0)
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    wmax = {"AB": 4, "C": 256, "D": 64}
    used = sorted(set(layer_classes))
    out = {}
    t_work = {}
    for label, threads, budget in (("all", cores, budgets[0]), ("1thread", 1, budgets[1])):
        per_class = {}
        t_start = time.perf_counter()
        with threadpool_limits(limits=threads):
            for cls in used:
                w = wmax[cls]
                cs = _sample_chi(chi, w, budget)
                (sc, ss), (zc, zs) = _time_oracle_step(cs, w, w, w, rng)
                fc, fs = _oracle_step_flops(cs, w, w, w)
                Fc, Fs = _oracle_step_flops(chi, w, w, w)
                zfc, zfs = _oracle_zip_flops(cs, w, w)
                Zfc, Zfs = _oracle_zip_flops(chi, w, w)
                per_class[cls] = {"step_s": sc * Fc / fc + ss * Fs / fs, "zip_s": zc * Zfc / zfc + zs * Zfs / zfs,
                                  "sample_chi": cs, "mpo_bond": w, "sample_seconds": sc + ss + zc + zs}
        t_work[label] = time.perf_counter() - t_start
        total = 0.0
        for cls, bonds in zip(layer_classes, bonds_per_layer):
            sat = sum(min(b, chi) ** 3 for b in bonds[1:-1]) / float(chi) ** 3
            pc = per_class[cls]
            total += sat * (pc["zip_s"] + sweeps * pc["step_s"])
        out[label] = {"value": len(layer_classes) / total, "threads": threads, "sample_seconds": round(t_work[label], 1),
                      "sample_chi": {c: v["sample_chi"] for c, v in per_class.items()},
                      "seconds_per_step_at_chi": {c: round(v["step_s"], 2) for c, v in per_class.items()},
                      "seconds_per_zip_step_at_chi": {c: round(v["zip_s"], 2) for c, v in per_class.items()}}
    return {"value": out["all"]["value"], "unit": "gate-layers/s", "cores": cores, "kind": "oracle",
            "value_1thread": out["1thread"]["value"],
            "sample": "per layer class (%s) of the timed layers: one oracle two-site step (local tensor, LAPACK "
                      "SVD, environment update) and one oracle zip-up step on random inputs at the class's "
                      "largest MPO bond and bond %s (all %d cores, %.1f s) or %s (1 thread, %.1f s); each part "
                      "scaled to chi=%d by the ratio of the oracle's operation counts; a layer = (n-1) zip-up "
                      "+ %d (n-1) two-site steps weighted by sum_k (chi_k/chi)^3 of the GPU run's bonds"
                      % ("/".join(used), out["all"]["sample_chi"], cores, t_work["all"],
                         out["1thread"]["sample_chi"], t_work["1thread"], chi, sweeps),
            "detail": out}


def layer_class(layer, n_rows_width=6):
    """A/B (horizontal couplers), C or D (vertical couplers, (r + c) even / odd) of a layer of
    the 54-qubit snake, from its two-qubit gates' chain sites."""
    two = [(q0, q1) for q0, q1, _ in layer if q1 >= 0]
    if not two:
        return "AB"
    q0, q1 = min(two[0]), max(two[0])
    if q1 - q0 == 1 and q0 // n_rows_width == q1 // n_rows_width:
        return "AB"
    r = q0 // n_rows_width
    c = q0 % n_rows_width if r % 2 == 0 else n_rows_width - 1 - q0 % n_rows_width
    return "C" if (r + c) % 2 == 0 else "D"


# ------------------------------------------------------------- extra legs
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
        out["K%d" % K] = {"gate_layers_per_s": steps / dt, "f_steps": fs, "F_tilde": st.fidelity()["F_tilde"],
                          "contraction_tflops": tflops(st.kernel_stats("contract"))}
        st.close()
    return out


def closed_leg(circuits, torch, n_amp):
    """Closed-mode amplitudes <x|U|0> of the 54-qubit circuit at chi = 64 (cut after layer 10,
    forward MPS built once, one backward MPS per bitstring), split precision."""
    import numpy as np
    from paper_2207_05612_amd import closed, mps
    c = circuits.sycamore_like_54_workload(0, depth=DEPTH)
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
            "F_tilde_forward": f_fwd, "abs_amplitudes": [abs(v) for v in vals]}


def batched_leg(mps, circuits, torch, count, sweeps, progress):
    """The first `count` instances of circuits.batched_instances(64), each on its own stream,
    one apply_layer_dmrg_batched call per layer over the instances still active; reported as
    instance-layers per second (a first untimed layer warms the kernels up)."""
    insts = circuits.batched_instances(64)[:count]
    streams = [torch.cuda.Stream() for _ in insts]
    states = [mps.MPS(c.n, None, max_chi=chi, precision=mps.MPS_BF16X3, stream=s.cuda_stream)
              for (c, chi), s in zip(insts, streams)]
    mps.apply_layer_dmrg_batched(states, [c.layers[0] for c, _ in insts], [chi for _, chi in insts], sweeps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    for d in range(1, max(len(c.layers) for c, _ in insts)):
        act = [i for i, (c, _) in enumerate(insts) if d < len(c.layers)]
        mps.apply_layer_dmrg_batched([states[i] for i in act], [insts[i][0].layers[d] for i in act],
                                     [insts[i][1] for i in act], sweeps)
        done += len(act)
        log(progress, "batched layer %d: %d instances" % (d, len(act)))
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    eps = [st.fidelity()["eps_tilde"] for st in states]
    for st in states:
        st.close()
    return {"instances": count, "instance_layers": done, "seconds": dt, "instance_layers_per_s": done / dt,
            "precision": "bf16x3", "n_sweeps": sweeps, "mean_eps_tilde": float(sum(eps) / len(eps)),
            "workload": "circuits.batched_instances(64)[:%d] (n 20..40, depth 8..20, chi 32..512, widths 4..6, "
                        "Haar), layers 1.. timed" % count}


def statevector_leg(mps, circuits, torch, n_qubits):
    """Gate passes of the exact statevector (HBM-bound: every pass reads and writes all 2^n
    FP64 complex amplitudes) on a Sycamore-layout circuit of n_qubits."""
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
        rec = json.load(open(SV_TRAFFIC_FILE))
        if rec.get("source_hash") == source_hash(("statevector.hip",)) and rec.get("n_qubits") == c.n:
            traffic = rec.get("bytes_per_launch")
    return {"n_qubits": c.n, "layers": len(c.layers) - 1, "gate_passes": passes, "ms": ms,
            "ms_per_pass": ms / passes,
            "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                         "algorithmic_bytes_per_launch": bytes_per_pass,
                         "kernel": "sv_2q_kernel, sv_2q_bit0_kernel (one two-qubit pass over all amplitudes)"}}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU: the compression step has no multi-GPU path "
              "(--gpus %d requested; the sharding design is written up, not built)" % args.gpus, file=sys.stderr)
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

    c = circuits.sycamore_like_54_workload(args.seed, depth=DEPTH)
    warmup = max(0, min(args.warmup, DEPTH - 1))
    steps = max(1, min(args.steps, DEPTH - warmup))
    prec_name = args.precision
    prec = getattr(mps, "MPS_" + prec_name.upper())
    run = run_layers(mps, c, prec, args.chi, args.sweeps, warmup, steps, torch, args.progress, args.samples,
                     keep=args.samples > 0)
    dt = sum(run["secs"])
    value = steps / dt
    stats = run["stats"]
    con = stats["contract"]
    achieved = tflops(con)
    peak = PEAK[prec_name]
    ratio = traffic_ratio(GEMM_KERNEL[prec_name].split("<")[0] if prec_name in ("bf16x3", "bf16x2")
                          else GEMM_KERNEL[prec_name], GEMM_SOURCE[prec_name])
    alg_bytes = con["bytes"] / max(con["launches"], 1)
    layers_timed = list(range(warmup, warmup + steps))
    classes = [layer_class(c.layers[d]) for d in layers_timed]

    gemm_roof = {"bound": "mfma", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                 "frac": achieved / peak,
                 "traffic": ratio * alg_bytes if ratio is not None else None,
                 "algorithmic_bytes_per_launch": alg_bytes,
                 "kernel": "%s (complex planar GEMM, %d launches, %.1f ms)"
                           % (GEMM_KERNEL[prec_name], con["launches"], con["ms"])}
    out = {
        "metric": "gate-layers/s & TFLOP/s at chi=1024, split-FP32 vs FP64 on 1 GPU, equal fidelity",
        "value": value,
        "unit": "gate-layers/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": dt * 1e3 / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[prec_name],
        "data": "synthetic",
        "config": {"workload": "54-qubit 6x9 snake, fSim + random 1q gates, depth %d, seed %d; layers %d..%d timed "
                               "(%d of %d requested; the circuit ends at layer %d)"
                               % (DEPTH, args.seed, layers_timed[0], layers_timed[-1], steps, args.steps, DEPTH - 1),
                   "chi": args.chi, "n_sweeps": args.sweeps, "contraction_precision": prec_name,
                   "truncation_precision": "fp64", "max_bond": max(run["bonds"]),
                   "layer_classes": "".join(x[0] if x != "AB" else "A" for x in classes)},
        "seconds_per_layer": [round(x, 3) for x in run["secs"]],
        "contraction_tflops": achieved,
        "all_kernels_algorithmic_tflops": sum(v["flops"] for v in stats.values()) / dt / 1e12,
        "time_split_ms": {k: round(v["ms"], 1) for k, v in stats.items()},
        "class_algorithmic_tflops": {k: round(tflops(v), 2) for k, v in stats.items() if v["flops"] > 0},
        "f_delta": run["f"],
        "F_tilde_after_timed_layers": run["fid"]["F_tilde"],
        "roofline": gemm_roof,
        "contraction_frac_of_fp32_mfma_peak": achieved / PEAK["fp32"],
        "roofline_contraction": dict(gemm_roof),
        "truncation_counters": run["counters"],
    }
    tri = stats["tridiag"]
    if tri["ms"] > 0:
        tri_tf = tflops(tri)
        tri_ratio = traffic_ratio("hetrd_kernel", ("hetrd.hip",))
        tri_bytes = tri["bytes"] / max(tri["launches"], 1)
        out["roofline_truncation"] = {
            "bound": "alu", "achieved": tri_tf, "peak": PEAK["fp64"], "unit": "TFLOP/s", "frac": tri_tf / PEAK["fp64"],
            "traffic": tri_ratio * tri_bytes if tri_ratio is not None else None,
            "algorithmic_bytes_per_launch": tri_bytes,
            "kernel": "hetrd_kernel (persistent FP64 tridiagonal reduction, %d launches, %.1f ms)"
                      % (tri["launches"], tri["ms"])}
        if tri["ms"] > con["ms"]:
            out["roofline"] = dict(out["roofline_truncation"])
        trunc_ms = sum(stats[k]["ms"] for k in ("gram", "tridiag", "eigh"))
        out["truncation_seconds"] = trunc_ms / 1e3
        out["truncation_effective_tflops"] = (
            # the truncation's algorithmic count: 320 chi'^3 FP64 flops per two-site step
            sum(320.0 * min(b, args.chi) ** 3 for bonds in run["bonds_per_layer"] for b in bonds[1:-1])
            * (1 + args.sweeps) / (trunc_ms * 1e-3) / 1e12 if trunc_ms > 0 else 0.0)
    if run["sampling"]:
        from paper_2207_05612_amd import analysis
        out["sampling"] = run["sampling"]
        st = run.pop("state")
        log(args.progress, "xeb against the sampled MPS")
        out["sampling"]["xeb_self"] = xeb_leg(analysis, st, st, args.samples, torch,
                                              "the sampled MPS itself (2^N sum_x p(x)^2 - 1)")
        if args.xeb_fp64:
            ref = run_layers(mps, c, mps.MPS_FP64, args.chi, args.sweeps, warmup, steps, torch, args.progress,
                             tag="xeb fp64 ", keep=True)["state"]
            out["sampling"]["xeb_fp64"] = xeb_leg(analysis, st, ref, args.samples, torch,
                                                  "the all-FP64 path's MPS over the same layers (the oracle's "
                                                  "arithmetic on the GPU; proxy for the oracle MPS)")
            ref.close()
        st.close()
    if args.fp64_steps and prec_name != "fp64":
        n64 = min(args.fp64_steps, steps)
        r64 = run_layers(mps, c, mps.MPS_FP64, args.chi, args.sweeps, warmup, n64, torch, args.progress,
                         tag="fp64 ")
        t_split = sum(run["secs"][:n64])
        t64 = sum(r64["secs"])
        out["fp64_path"] = {"value": n64 / t64, "unit": "gate-layers/s", "layers": "%d..%d" % (warmup, warmup + n64 - 1),
                            "seconds_per_layer": [round(x, 3) for x in r64["secs"]],
                            "contraction_tflops": tflops(r64["stats"]["contract"]),
                            "time_split_ms": {k: round(v["ms"], 1) for k, v in r64["stats"].items()},
                            "f_delta": r64["f"]}
        out["speedup_vs_fp64"] = t64 / t_split
        out["max_rel_f_delta_diff_vs_fp64"] = max(abs(a - b) / b for a, b in zip(run["f"][:n64], r64["f"]))
    if args.single_site:
        ss = {}
        for name, pr in (("split", prec), ("fp64", mps.MPS_FP64)):
            r = run_layers(mps, c, pr, args.chi, args.sweeps, warmup, steps, torch, args.progress,
                           update="single-site", tag="single-site %s " % name)
            ss[name] = {"value": steps / sum(r["secs"]), "f_delta": r["f"],
                        "contraction_tflops": tflops(r["stats"]["contract"])}
        out["single_site"] = {"update": "single-site sweeps after the same zip-up (the paper's update rule)",
                              "value": ss["split"]["value"], "unit": "gate-layers/s",
                              "speedup_vs_fp64_single_site": ss["split"]["value"] / ss["fp64"]["value"],
                              "split": ss["split"], "fp64": ss["fp64"]}
    if args.multilayer_chi:
        out["multilayer"] = multilayer_leg(mps, c, prec, args.multilayer_chi, args.sweeps, warmup, min(4, steps),
                                           torch)
    if args.closed_amplitudes:
        out["closed"] = closed_leg(circuits, torch, args.closed_amplitudes)
    if args.statevector:
        out["statevector"] = statevector_leg(mps, circuits, torch, args.statevector)
    if args.batched:
        out["batched"] = batched_leg(mps, circuits, torch, args.batched, args.sweeps, args.progress)
    if args.cpu_baseline:
        log(args.progress, "cpu baseline")
        out["cpu_baseline"] = cpu_baseline(args.chi, c.n, args.sweeps, classes, run["bonds_per_layer"])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
