"""Benchmark of the compressed stage loop on one MI355X.

Workload (the headline configuration, the largest that lives in one GPU's
HBM): 33-qubit random circuit, depth 16 (per layer U3 with seeded angles on
every qubit, then CZ on 8 disjoint seeded pairs; 656 gates), complex64
state (64 GiB uncompressed), 2^24-amplitude SV blocks, LOG-domain codec with
eb = 1e-5, fused dense operations of up to 5 qubits on the FP32 matrix
cores, whole compressed state in HBM.  `--workload qft` runs the 30-qubit
QFT on an Ry product state (2^22-amplitude blocks, 4-qubit fusion).

One step = reset to |0...0> + every stage of the circuit through
stage_apply_compressed (decode -> apply fused gates -> re-encode per tile).
The timed region holds exactly K steps, bracketed by device synchronisation.
Result check (after the timed region): the random circuit's inverse is run
on the final state, so F^2 = |psi(0)|^2 / |psi|^2 is exact; the QFT is
checked on sampled amplitudes against its closed form.

Metric: amplitude*gates/s = 2^n * (circuit gates) / step time.
Roofline: the pass kernel is HBM-bound; its algorithmic bytes per stage are
the compressed records read and written plus the chunk directory read and
written.  Achieved GB/s = those bytes / the stages' kernel time, both taken
from HIP events recorded on the library's stream inside the timed steps.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
VALU_PEAK_LANE_OPS = 256 * 4 * 32 * 2.4e9     # CUs x SIMDs x 32-bit lanes per clock x clock: FP32 vector 157.3 TFLOP/s / 2
METRIC = "compressed-SV amplitude·gates/s, GB/s vs HBM peak at fidelity≥0.99; compression ratio"


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="random",
                    choices=["random", "qft", "random-mirror", "batch", "qaoa-spill", "pipeline"],
                    help="random: random U3/CZ layers (default, 33 qubits, depth 16); qft: QFT on an Ry product "
                         "(30 qubits); random-mirror: the random layers followed by their inverse, timed "
                         "together; batch: 512 uneven circuits of "
                         "18-26 qubits run together (sv_batch_apply) and one after another; qaoa-spill: "
                         "QAOA ring p=3 (32 qubits) with the device pools capped so records spill to a "
                         "pinned host pool, against the same run on the device only; pipeline: the 30-qubit QFT "
                         "with the compressed state in pinned host memory, each stage's groups copied through the "
                         "GPU on S = 1, 2, 4, 8 streams (sv_pipe_*), against the device-resident run")
    ap.add_argument("--pool-frac", type=float, default=0.25,
                    help="qaoa-spill: device pool capacity per state copy, as a fraction of the "
                         "uncompressed complex64 size")
    ap.add_argument("--device-pool-gb", type=float, default=0.0,
                    help="qaoa-spill: device pool capacity per state copy in GB (instead of --pool-frac); "
                         "with it the device-only run is skipped (for states whose records exceed the HBM)")
    ap.add_argument("--host-pool-gb", type=float, default=0.0,
                    help="qaoa-spill: pinned host pool in GB, both state copies together (default: twice "
                         "the uncompressed complex64 size)")
    ap.add_argument("--batch-count", type=int, default=512)
    ap.add_argument("--n", type=int, default=0, help="qubits (default: 33 for random, 30 for qft)")
    ap.add_argument("--flags", type=int, default=None,
                    help="sv_config_t flags (1 no scratch, 2 no MFMA, 4 one stage per gate, 8 diagonal-free, "
                         "16 commutation-aware, 32 group-sized scratch; default 32, batch workload 1)")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--domain", choices=["log", "lin", "raw"], default="log",
                    help="codec domain of the qft / random-mirror workloads (default log; raw = no compression)")
    ap.add_argument("--eb", type=float, default=0.0, help="codec error bound (default 1e-5)")
    ap.add_argument("--fuse", type=int, default=0, help="fusion width (default 4 for qft, 5 for random-mirror)")
    ap.add_argument("--host-resident", action="store_true",
                    help="qft / random-mirror: 64 MiB device pools, so that the records live in a pinned host "
                         "pool that the kernels read and write over the host link")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batch", action="store_true",
                    help="random workload: skip the batched 512-circuit sub-line")
    ap.add_argument("--no-predictor-pools", action="store_true",
                    help="random workload: worst-case device pools instead of pools sized by the predictor")
    ap.add_argument("--no-autotune", action="store_true",
                    help="random workload: no tile / fusion autotuning (fusion width 5 unless --fuse)")
    ap.add_argument("--no-variant", action="store_true",
                    help="skip the diagonal-free planner variant (profiles of the headline launches only)")
    ap.add_argument("--cpu-n", type=int, default=0,
                    help="qubits of the CPU-baseline sample (default 30: the headline's generator and global-qubit count)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="CPU baseline: stop after the stage that passes this much oracle time")
    ap.add_argument("--variant-steps", type=int, default=3, help="timed steps of the planner variant")
    ap.add_argument("--stats-out", default="")
    ap.add_argument("--persistent", action="store_true",
                    help="also time the whole-circuit queue launch (sv_persistent_apply) and report it beside")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (HBM counter calibration) and exit")
    return ap.parse_args()


def progress(msg):
    """A progress line on stderr (the result is the one JSON line on stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def copy_calibration():
    """A plain device-to-device copy of 1 GiB, three times: the reference
    for scaling the FETCH_SIZE / WRITE_SIZE counters to bytes."""
    import torch
    n = (1 << 30) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "copies": 3}))


def qft_ry_closed_form(n, theta, idx):
    """Amplitudes of the QFT (no final swaps) of the product state
    (x) Ry(theta_q)|0>: psi(y) = 2^(-n/2) prod_i (cos(theta_i/2) +
    sin(theta_i/2) exp(2 pi i frac(2^i rev_n(y) / 2^n)))."""
    import numpy as np
    idx = np.asarray(idx, dtype=np.uint64)
    rev = np.zeros_like(idx)
    for b in range(n):
        rev |= ((idx >> np.uint64(b)) & np.uint64(1)) << np.uint64(n - 1 - b)
    mask = np.uint64((1 << n) - 1)
    acc = np.ones(idx.size, dtype=np.complex128)
    for i in range(n):
        num = (rev << np.uint64(i)) & mask
        ph = 2.0 * np.pi * num.astype(np.float64) / float(1 << n)
        acc *= np.cos(theta[i] / 2) + np.sin(theta[i] / 2) * np.exp(1j * ph)
    return acc * 2.0 ** (-0.5 * n)


# committed counter profiles of the pass kernel, per default workload:
# (n, tile, fuse, flags) they were taken at and the file stem
PROFILES = {"random": ((33, 12, 3, 32), "pass_kernel_random33"),
            "qft": ((30, 12, 4, 32), "pass_kernel_qft30")}


def _profile_field(workload, key, n, tile, fuse, flags, field):
    """A figure from a committed counter profile, or None when the run
    differs from the profiled one or the kernel source changed since."""
    import hashlib
    import re
    if workload not in PROFILES or PROFILES[workload][0] != (n, tile or 12, fuse, flags):
        return None
    prof = os.path.join(ROOT, "profiles", f"{PROFILES[workload][1]}_{key}.md")
    src = os.path.join(ROOT, "paper_2410_14088_amd", "csrc", "bmq_kernels.hip")
    try:
        text = open(prof).read()
        sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    except OSError:
        return None
    m_sha = re.search(r"^kernel_sha256: ([0-9a-f]{64})$", text, re.M)
    m_val = re.search(rf"^{field}: ([0-9.e+]+)$", text, re.M)
    if not m_sha or not m_val or m_sha.group(1) != sha:
        return None
    return float(m_val.group(1))


def counter_traffic(n, tile, fuse, flags=0, workload="random"):
    """HBM bytes per pass-kernel launch (FETCH_SIZE + WRITE_SIZE profile)."""
    v = _profile_field(workload, "hbm_counters", n, tile, fuse, flags, "traffic_bytes_per_launch")
    return None if v is None else int(v)


def valu_profile(n, tile, fuse, flags=0, workload="random"):
    """Issued VALU lane-operations per second of the pass kernel and their
    fraction of the 32-bit VALU ceiling (SQ-counter profile)."""
    ops = _profile_field(workload, "sq_counters", n, tile, fuse, flags, "valu_lane_ops_per_s")
    if ops is None:
        return None
    return {"bound": "alu", "achieved": ops, "peak": VALU_PEAK_LANE_OPS, "unit": "lane-op/s",
            "frac": ops / VALU_PEAK_LANE_OPS, "source": "issued VALU instructions (SQ counters), not algorithmic"}


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(workload: str, n: int, seconds: float):
    """The oracle as it stands, on the host's cores: per stage of the same
    circuit generator (at n qubits, with the headline's number of global
    qubits), decode every SV block with the CPU codec, apply the stage's
    gates in FP64 (OpenMP), re-encode every block; the blocks' codec calls
    run on a thread per core.  Stops after the stage that passes `seconds`
    and reports amplitude*gates/s over the stages it ran, with the codec's
    own rate (uncompressed float32 bytes decoded and encoded per second)."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np
    from oracle import native as N
    from oracle import planner as OP
    from paper_2410_14088_amd import circuits as C

    if workload == "qft":
        d = C.config(1, n=n)
        b = n - 8                      # 8 global qubits, as at 30 qubits
    else:
        d = C.config(2, n=n)
        b = n - 9                      # 9 global qubits, as at 33 qubits
    gates = d["gates"]
    stages = OP.partition(gates, b, 2)
    nb = 1 << (n - b)
    blk = 1 << b
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count()
    pool = ThreadPoolExecutor(max_workers=threads)
    zero = np.zeros(blk, np.float32)
    one = zero.copy()
    one[0] = 1.0
    streams = [N.encode_block(one if k == 0 else zero, zero, d["domain"], d["eb"]) for k in range(nb)]
    done_gates = 0
    ran = 0
    t_dec = t_app = t_enc = 0.0
    t0 = time.perf_counter()
    for s0, s1 in stages:
        psi = np.empty(1 << n, dtype=np.complex128)

        def dec(k):
            r, i = N.decode_block(streams[k], blk)
            psi[k * blk:(k + 1) * blk] = r.astype(np.float64) + 1j * i.astype(np.float64)
        ta = time.perf_counter()
        list(pool.map(dec, range(nb)))
        tb = time.perf_counter()
        psi = N.apply_circuit(psi, n, gates[s0:s1])
        tc = time.perf_counter()

        def enc(k):
            v = psi[k * blk:(k + 1) * blk]
            return N.encode_block(v.real.astype(np.float32), v.imag.astype(np.float32), d["domain"], d["eb"])
        streams = list(pool.map(enc, range(nb)))
        td = time.perf_counter()
        t_dec += tb - ta
        t_app += tc - tb
        t_enc += td - tc
        done_gates += s1 - s0
        ran += 1
        del psi
        progress(f"cpu baseline: stage {ran} of {len(stages)} done ({time.perf_counter() - t0:.1f} s)")
        if time.perf_counter() - t0 >= seconds:
            break
    dt = time.perf_counter() - t0
    pool.shutdown()
    name = "QFT on the same Ry product" if workload == "qft" else "random U3/CZ layers of the same generator"
    fbytes = ran * (8 << n)            # float32 re + im per amplitude, per stage
    return dict(value=(2 ** n) * done_gates / dt, unit="amplitude·gates/s", cores=threads, kind="oracle",
                cpu=cpu_model(), nproc=os.cpu_count(),
                codec_decode_gbps=fbytes / t_dec / 1e9, codec_encode_gbps=fbytes / t_enc / 1e9,
                fp64_apply_amp_gates_per_s=(2 ** n) * done_gates / t_app,
                seconds={"decode": t_dec, "apply": t_app, "encode": t_enc},
                sample=f"{n}-qubit {name}: first {ran} of {len(stages)} stages ({done_gates} of {len(gates)} "
                       f"gates), 2^{b}-amplitude blocks, LOG eb={d['eb']}: CPU codec decode/encode of every "
                       f"block per stage ({threads} threads) + FP64 OpenMP gate application, {dt:.1f} s")


def batch_planning(mix, flags, fuse, train=32, margin=0.1, budget_frac=0.5, seed=11):
    """Memory planning for a batch: the block predictor, trained online on the
    first `train` circuits (planning features before each stage, labels after
    it), is rolled over every circuit's plan to predict its peak compressed
    size; circuits are admitted under a device budget of budget_frac of the
    worst-case arenas, with pools sized by the prediction, against worst-case
    pools (no predictor) and the size a circuit has before it runs.  The
    admitted circuits then run in one batched launch with their predicted
    pools; a circuit whose pools overflow is re-run with worst-case pools.
    Returns the figures and the run's record bytes per circuit."""
    import numpy as np
    import torch
    from paper_2410_14088_amd import bmq
    from paper_2410_14088_amd import circuits as C

    def cfg_of(d, pool=0):
        return bmq.Config(n=d["n"], b=d["n"] - 8, inner=2, fuse=fuse, domain=1, eb=1e-5, flags=flags,
                          pool_bytes=int(pool))
    t0 = time.perf_counter()
    # online training, stage by stage, on the first circuits (planning
    # features before a stage, labels after it), and their actual peaks
    pred = bmq.Predictor(C.mlp_init_params(seed), "cuda:0", lr=2e-3)
    train_peaks, train_plans = [], []
    loss = None
    for d in mix[:train]:
        c = cfg_of(d)
        plan = bmq.Plan(d["gates"], c)
        sv = bmq.State(c, "cuda:0")
        peak = 0.0
        for s in range(plan.n_stages):
            X = sv.plan_features(plan, s)
            sv.apply(plan, s, 1)
            y, mode = sv.plan_labels()
            for _ in range(4):
                loss = pred.train_step(X, y, mode)
            peak = max(peak, float(torch.exp2(y.double() + c.b).sum()))
        train_peaks.append(peak)
        train_plans.append(plan)
        sv.close()
    loss = float(loss.item())
    progress(f"batch planning: predictor trained on {train} circuits")
    # calibration on the training circuits: the largest actual / predicted peak
    tp = np.array([float(bmq.predict_bytes(pred.params, p).max()) for p in train_plans])
    calib = max(1.0, float(np.max(np.array(train_peaks) / tp)))
    t_train = time.perf_counter() - t0
    rest = mix[train:]
    cfgs = [cfg_of(d) for d in rest]
    plans = [bmq.Plan(d["gates"], c) for d, c in zip(rest, cfgs)]
    t0 = time.perf_counter()
    raw = np.array([float(bmq.predict_bytes(pred.params, p).max()) for p in plans])
    peaks = raw * calib
    t_pred = time.perf_counter() - t0
    init = np.array([8.0 * (1 << (d["n"] - 6)) + 8.0 for d in rest])       # |0...0>: headers + one record
    worst_all = int(bmq.admit(cfgs, None, margin, 1 << 62)[2].sum())
    budget = int(budget_frac * worst_all)
    adm_w = bmq.admit(cfgs, None, margin, budget)[0]
    adm_p, pool_p, arena_p = bmq.admit(cfgs, peaks, margin, budget)
    adm_i = bmq.admit(cfgs, init, margin, budget)[0]
    pred_all = int(bmq.admit(cfgs, peaks, margin, 1 << 62)[2].sum())
    # run the predicted-pool admitted set, batched; overflowing circuits are re-run
    idx = list(np.flatnonzero(adm_p))
    states = [bmq.State(cfg_of(rest[i], pool_p[i]), "cuda:0") for i in idx]
    fallback = []
    try:
        bmq.batch_apply(states, [plans[i] for i in idx])
    except bmq.BmqError as e:
        if e.code != -3:
            raise
    torch.cuda.synchronize()
    final = []
    for k, (i, st) in enumerate(zip(idx, states)):
        try:
            rec = st.footprint()[0]
        except bmq.BmqError:
            st.close()
            st = bmq.State(cfg_of(rest[i]), "cuda:0")
            st.apply(plans[i])
            rec = st.footprint()[0]
            fallback.append(int(i))
        # the final state's stream bytes (records + headers) against the prediction
        final.append((rec + 8 * (1 << (rest[i]["n"] - 6))) / peaks[i])
        st.close()
    torch.cuda.empty_cache()
    return {
        "train_circuits": train, "planned_circuits": len(rest), "margin": margin,
        "budget_bytes": budget, "budget_fraction_of_worst_case": budget_frac,
        "admitted_worst_case_pools": int(adm_w.sum()), "admitted_predicted_pools": int(adm_p.sum()),
        "admitted_before_run_size": int(adm_i.sum()),
        "device_bytes_all_worst_case": worst_all, "device_bytes_all_predicted": pred_all,
        "fallbacks_to_worst_case": len(fallback), "train_s": t_train, "predict_s": t_pred,
        "train_loss": loss, "calibration": calib,
        "final_over_predicted_peak_median": float(np.median(final)) if final else None,
        "final_over_predicted_peak_max": float(np.max(final)) if final else None,
    }


def bench_batch(args):
    """Many independent circuits: the batched launch against the per-circuit
    loop on the same states and plans (identical records either way), and
    the predictor's memory planning (admission under a device budget)."""
    out = batch_line(args)
    print(json.dumps(out))


def batch_line(args, planning=True):
    import torch
    from paper_2410_14088_amd import bmq
    from paper_2410_14088_amd import circuits as C
    mix = C.batch_mix(args.batch_count)
    flags = args.flags if args.flags_given and args.flags else 1   # no scratch planes: 512 arenas fit together
    fuse = args.fuse if args.workload == "batch" and args.fuse else 4
    states, plans, amp_gates = [], [], 0
    for d in mix:
        cfg = bmq.Config(n=d["n"], b=d["n"] - 8, inner=2, fuse=fuse, domain=1, eb=1e-5, flags=flags)
        plans.append(bmq.Plan(d["gates"], cfg))
        states.append(bmq.State(cfg, "cuda:0"))
        amp_gates += (1 << d["n"]) * len(d["gates"])
    res = {}
    for mode in ["batched"] * args.warmup + ["batched", "sequential"] + ["persistent"] * (args.warmup + 1):
        for st in states:
            st.reset()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if mode == "batched":
            bmq.batch_apply(states, plans)
        elif mode == "persistent":
            bmq.persistent_apply(states, plans)
        else:
            for st, p in zip(states, plans):
                st.apply(p)
        torch.cuda.synchronize()
        res[mode] = time.perf_counter() - t0
        progress(f"batch {mode}: {res[mode] * 1e3:.1f} ms")
    fp = sum(st.footprint()[0] for st in states)
    for st in states:
        st.close()
    del states
    torch.cuda.empty_cache()
    out = {
        "metric": METRIC, "value": amp_gates / res["batched"], "unit": "amplitude·gates/s", "n_gpus": 1,
        "steps": 1, "warmup": args.warmup, "ms_per_step": res["batched"] * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batch-{len(mix)}-circuits-18-26q", "circuits": len(mix),
                   "amplitudes": sum(1 << d["n"] for d in mix), "amp_gates": amp_gates, "domain": "log",
                   "eb": 1e-5, "fuse_qubits": fuse, "flags": flags, "block_qubits": "n-8"},
        "sequential_value": amp_gates / res["sequential"], "sequential_ms": res["sequential"] * 1e3,
        "speedup_vs_sequential": res["sequential"] / res["batched"],
        "persistent_ms": res["persistent"] * 1e3,
        "persistent_value": amp_gates / res["persistent"],
        "compression_ratio_vs_complex64": sum(8 << d["n"] for d in mix) / fp,
    }
    if planning:
        out["planning"] = batch_planning(mix, flags, fuse)
    return out


def headline_pools(plan, n, b, fuse, tile, flags, eb, margin=0.1, seed=11):
    """Memory planning for the headline (Section 4.4 with the learned
    predictor): the block predictor is trained online on three smaller
    circuits of the same generator and global-qubit count (planning features
    before each stage, labels after it), calibrated by their largest actual /
    predicted peak, and rolled over the headline's plan; the predicted peak
    sizes the device pools (sv_admit, 10 % margin) instead of the worst case."""
    import torch
    from paper_2410_14088_amd import bmq
    from paper_2410_14088_amd import circuits as C
    t0 = time.perf_counter()
    c = n - b
    pred = bmq.Predictor(C.mlp_init_params(seed), "cuda:0", lr=2e-3)
    trained = []
    for tn, sd in ((21, 101), (22, 102), (23, 103)):
        cfg = bmq.Config(n=tn, b=tn - c, inner=2, fuse=fuse, domain=1, eb=eb, tile=tile, flags=flags)
        tplan = bmq.Plan(C.random_layers(tn, 16, sd), cfg)
        sv = bmq.State(cfg, "cuda:0")
        peak = 0.0
        for st in range(tplan.n_stages):
            X = sv.plan_features(tplan, st)
            sv.apply(tplan, st, 1)
            y, mode = sv.plan_labels()
            for _ in range(4):
                pred.train_step(X, y, mode)
            peak = max(peak, float(torch.exp2(y.double() + cfg.b).sum()))
        sv.close()
        trained.append((peak, tplan))
    # calibration: the largest actual / predicted peak of the training circuits
    ratios = [pk / float(bmq.predict_bytes(pred.params, pl).max()) for pk, pl in trained]
    calib = max(ratios)
    raw = float(bmq.predict_bytes(pred.params, plan).max())
    hcfg = bmq.Config(n=n, b=b, inner=2, fuse=fuse, domain=1, eb=eb, tile=tile, flags=flags)
    _, pools, arenas = bmq.admit([hcfg], [raw * calib], margin, 1 << 62)
    _, wpools, warenas = bmq.admit([hcfg], None, margin, 1 << 62)
    torch.cuda.empty_cache()
    out = {"trained_on": "random U3/CZ layers, depth 16, 21-23 qubits, 9 global qubits (seeds 101-103)",
           "calibration": calib, "training_actual_over_predicted": ratios,
           "predicted_peak_stream_bytes": raw * calib, "margin": margin,
           "pool_bytes": int(pools[0]), "arena_bytes": int(arenas[0]),
           "worst_case_pool_bytes": int(wpools[0]), "worst_case_arena_bytes": int(warenas[0]),
           "host_pool_bytes": 8 << 30,
           "seconds": time.perf_counter() - t0}
    progress(f"memory planning: predicted peak {raw * calib / 1e9:.1f} GB, pools {int(pools[0]) / 1e9:.1f} GB "
             f"(worst case {int(wpools[0]) / 1e9:.1f} GB)")
    return out


def autotune_headline(d, gates, args, inner=(2,), fuse=(2, 3, 4, 5), tiles=(12, 13)):
    """sv_autotune_space over tile sizes and fusion widths (or inner sizes)
    on the circuit's first four layers; the winner is used for the full
    circuit."""
    import torch
    from paper_2410_14088_amd import bmq
    n = d["n"]
    probe = 4 * (n + 8)                        # four layers: U3 on every qubit + 8 CZ
    cfg = bmq.Config(n=n, b=d["b"], inner=inner[0], fuse=fuse[0], domain=1, eb=d["eb"],
                     tile=args.tile or tiles[0], flags=args.flags)
    t0 = time.perf_counter()
    tl = (args.tile,) if args.tile else tiles
    progress(f"autotune: tiles {tl} x fusion {fuse} x inner {inner} on the first {probe} gates")
    best, table = bmq.autotune_space(gates, cfg, tiles=tl, fuse=fuse, inner=inner, probe_gates=probe)
    torch.cuda.empty_cache()
    # candidates within 1 % of the fastest are a tie (run-to-run spread):
    # take the widest fusion, then the smallest tile, among them
    fastest = min(table.values())
    tied = [k for k, v in table.items() if v <= 1.01 * fastest]
    t_, f_, m_ = sorted(tied, key=lambda k: (-k[2], -k[1], k[0]))[0] if len(inner) > 1 else \
        sorted(tied, key=lambda k: (-k[1], k[0]))[0]
    best = bmq.Config(n=best.n, b=best.b, inner=m_, fuse=f_, domain=best.domain, eb=best.eb, tile=t_,
                      pool_bytes=best.pool_bytes, flags=best.flags)
    progress(f"autotune: tile {best.tile}, fusion {best.fuse}, inner {best.inner} "
             f"({time.perf_counter() - t0:.1f} s)")
    return {"probe_gates": probe, "seconds": time.perf_counter() - t0,
            "ms": {f"tile{t}_fuse{f}_inner{m}": v for (t, f, m), v in sorted(table.items())},
            "chosen": {"tile_qubits": best.tile, "fuse_qubits": best.fuse, "inner_size": best.inner}}


def qaoa_ring_closed_form(n, gammas, betas, xs):
    """<x| prod_l RX(beta_l)^n RZZ_ring(gamma_l) H^n |0> for each x: a sum over
    Z-basis worldlines per site, contracted around the ring as the trace of a
    product of 2^p x 2^p transfer matrices (batched over the samples)."""
    import numpy as np
    p = len(gammas)
    W = 1 << p
    bits = [(np.arange(W) >> l) & 1 for l in range(p)]
    ang = np.zeros((W, W))
    for l in range(p):
        s_w = 1 - 2 * bits[l]
        ang += -gammas[l] / 2 * np.outer(s_w, s_w)
    bond = np.exp(1j * ang)
    def rx(b):
        c, s_ = np.cos(b / 2), np.sin(b / 2)
        return np.array([[c, -1j * s_], [-1j * s_, c]])
    R = [rx(b) for b in betas]
    site = np.ones((2, W), dtype=np.complex128)        # site factor for x_i = 0, 1
    for xi in (0, 1):
        for l in range(p):
            dst = bits[l + 1] if l + 1 < p else np.full(W, xi)
            site[xi] *= R[l][dst, bits[l]]
    xs = np.asarray(xs, dtype=np.uint64)
    T = np.broadcast_to(np.eye(W, dtype=np.complex128), (xs.size, W, W)).copy()
    for i in range(n):
        xi = ((xs >> np.uint64(i)) & np.uint64(1)).astype(np.int64)
        T = T @ (site[xi][:, :, None] * bond[None, :, :])
    return np.trace(T, axis1=1, axis2=2) / 2 ** (n / 2)


def bench_qaoa_spill(args):
    """Two-level memory at scale: the same QAOA run with device pools large
    enough and with capped device pools plus a pinned host pool."""
    import numpy as np
    import torch
    from paper_2410_14088_amd import bmq
    from paper_2410_14088_amd import circuits as C
    n = args.n or 32
    gates, gammas, betas = C.qaoa_ring(n, 3, 1003)
    res = {}
    rng = np.random.default_rng(7)
    idx = rng.integers(0, 1 << n, 512).astype(np.uint64)
    want = qaoa_ring_closed_form(n, gammas, betas, idx)
    large = args.device_pool_gb > 0
    # scratch-free at the default size; group-sized scratch planes when the
    # device pools are given explicitly (the state is then beyond the HBM)
    flags = bmq.SV_FLAG_GROUP_SCRATCH if large else bmq.SV_FLAG_NO_SCRATCH
    for mode in (("spill",) if large else ("device", "spill")):
        if mode == "device":
            pool = 0
        elif large:
            pool = int(args.device_pool_gb * 1e9) & ~255
        else:
            pool = int(args.pool_frac * (8 << n)) & ~255
        cfg = bmq.Config(n=n, b=n - 8, inner=2, fuse=args.fuse or 4, domain=1, eb=1e-5, pool_bytes=pool,
                         flags=flags)
        plan = bmq.Plan(gates, cfg)
        progress(f"qaoa {n} qubits, {mode}: {len(gates)} gates, {plan.n_stages} stages, device pool "
                 f"{pool / 1e9:.1f} GB per copy")
        sv = bmq.State(cfg, "cuda:0")
        if mode == "spill":
            hb = int(args.host_pool_gb * 1e9) & ~255 if args.host_pool_gb > 0 else 2 * (8 << n)
            sv.attach_host_pool(hb, exact=large)
            progress(f"host pool {hb / 1e9:.1f} GB attached")
        for _ in range(args.warmup):
            sv.reset()
            sv.apply(plan)
        torch.cuda.synchronize()
        sv.reset()
        t0 = time.perf_counter()
        if large:
            # stage by stage, with a progress line each (a stage moves a
            # large share of the records over the host link)
            st = []
            for s in range(plan.n_stages):
                st += sv.apply(plan, first=s, count=1, stats=True)
                progress(f"stage {s + 1}/{plan.n_stages}: records {st[-1]['bytes_out'] / 1e9:.1f} GB, "
                         f"{st[-1]['bytes_out_host'] / 1e9:.1f} GB of them on the host, "
                         f"{time.perf_counter() - t0:.1f} s")
        else:
            st = sv.apply(plan, stats=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        progress(f"{mode}: {dt:.1f} s")
        got = sv.amplitudes(torch.from_numpy(idx.astype(np.int64))).cpu().numpy().astype(np.complex128)
        f2 = abs(np.vdot(want, got)) ** 2 / (np.vdot(want, want).real * np.vdot(got, got).real)
        rec, host, _ = sv.footprint()
        res[mode] = dict(ms=dt * 1e3, value=(2 ** n) * len(gates) / dt, fidelity_f2_sampled=f2,
                         max_abs_err_sampled=float(np.abs(got - want).max()), record_bytes=rec, host_bytes=host,
                         peak_host_bytes=max(s["bytes_out_host"] for s in st), device_pool_bytes=pool or None,
                         stages=len(st))
        sv.close()
        del sv
        torch.cuda.empty_cache()
    out = {
        "metric": METRIC, "value": res["spill"]["value"], "unit": "amplitude·gates/s", "n_gpus": 1, "steps": 1,
        "warmup": args.warmup, "ms_per_step": res["spill"]["ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"qaoa-ring-{n}q-p3-host-spill", "n_qubits": n, "gates": len(gates),
                   "block_qubits": n - 8, "domain": "log", "eb": 1e-5, "fuse_qubits": args.fuse or 4,
                   "flags": flags, "device_pool_frac": None if large else args.pool_frac,
                   "device_pool_bytes": res["spill"]["device_pool_bytes"]},
        "spill": res["spill"], "device_only": res.get("device"),
        "compression_ratio_vs_complex64": (8 << n) / res["spill"]["record_bytes"],
    }
    print(json.dumps(out))


def bench_pipeline(args):
    """Host-resident state through the pipeline: one run per stream count,
    timed from |0...0> over every stage (host clock, each stage ends when
    its images are back in the host store), against the device-resident
    stage loop on the same plan; records compared after each run."""
    import numpy as np
    import torch
    from paper_2410_14088_amd import bmq
    from paper_2410_14088_amd import circuits as C
    n = args.n or 30
    d = C.config(1, n=n)
    gates = d["gates"]
    fuse = args.fuse or 4
    cfg = bmq.Config(n=n, b=d["b"], inner=2, fuse=fuse, domain=1, eb=d["eb"], flags=bmq.SV_FLAG_GROUP_SCRATCH)
    plan = bmq.Plan(gates, cfg)
    G = len(gates)
    sv = bmq.State(cfg, "cuda:0")
    for _ in range(max(1, args.warmup)):
        sv.reset()
        sv.apply(plan)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sv.reset()
        sv.apply(plan)
    torch.cuda.synchronize()
    dev_ms = (time.perf_counter() - t0) * 1e3 / args.steps
    progress(f"pipeline: device-resident {dev_ms:.1f} ms per run")
    ref_blocks = [sv.block_stream(k) for k in range(0, sv.n_blocks, max(1, sv.n_blocks // 16))]
    rng = np.random.default_rng(1)
    idx = rng.integers(0, 1 << n, 4096).astype(np.uint64)
    want = qft_ry_closed_form(n, d["thetas"], idx)
    runs = {}
    for S in (1, 2, 4, 8):
        pipe = bmq.Pipe(cfg, streams=S)
        pipe.apply(plan)                                   # warm-up
        best = None
        for _ in range(args.steps):
            pipe.reset()
            t0 = time.perf_counter()
            st = pipe.apply(plan, stats=True)
            dt = time.perf_counter() - t0
            best = dt if best is None or dt < best else best
        fp = pipe.footprint()
        sv.reset()
        pipe.load(sv)
        same = all(sv.block_stream(k) == ref_blocks[i]
                   for i, k in enumerate(range(0, sv.n_blocks, max(1, sv.n_blocks // 16))))
        got = sv.amplitudes(torch.from_numpy(idx.astype(np.int64))).cpu().numpy().astype(np.complex128)
        f2 = float(abs(np.vdot(want, got)) ** 2 / (np.vdot(want, want).real * np.vdot(got, got).real))
        moved = fp["h2d_bytes"] + fp["d2h_bytes"]
        runs[str(S)] = {"ms_per_step": best * 1e3, "value": (2 ** n) * G / best, "h2d_bytes": fp["h2d_bytes"],
                        "d2h_bytes": fp["d2h_bytes"], "host_link_gbps": moved / best / 1e9,
                        "host_store_bytes": fp["host_used"], "record_bytes": fp["record_bytes"],
                        "records_equal_device_run": same, "fidelity_f2_sampled": f2,
                        "slowest_stage_ms": max(s["ms"] for s in st)}
        progress(f"pipeline: {S} streams {best * 1e3:.1f} ms per run, {moved / best / 1e9:.1f} GB/s over the host link")
        pipe.close()
        del pipe
        torch.cuda.empty_cache()
    best_s = min(runs, key=lambda k: runs[k]["ms_per_step"])
    out = {
        "metric": METRIC, "value": runs[best_s]["value"], "unit": "amplitude·gates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": runs[best_s]["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"qft-on-ry-{n}q-host-resident-pipeline", "n_qubits": n, "block_qubits": d["b"],
                   "gates": G, "stages": plan.n_stages, "domain": "log", "eb": d["eb"], "fuse_qubits": fuse,
                   "streams": int(best_s)},
        "streams": runs, "device_resident_ms": dev_ms,
        "note": "host-link-inclusive rates: the state lives in pinned host memory between stages",
    }
    print(json.dumps(out))


def main():
    args = parse()
    args.fuse_given = bool(args.fuse)
    args.flags_given = args.flags is not None
    if args.flags is None:
        # scratch planes sized for one SV group (multi-pass stages run group by group)
        args.flags = 0 if args.workload == "batch" else 32
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); multi-GPU sharding of the "
              "stage loop is a design note, not implemented", file=sys.stderr)
        sys.exit(2)
    if args.workload == "qaoa-spill":
        bench_qaoa_spill(args)
        return
    if args.workload == "pipeline":
        bench_pipeline(args)
        return
    if args.workload == "batch" and not args.copy_calibration:
        bench_batch(args)
        return
    if args.copy_calibration:
        copy_calibration()
        return
    import math

    import numpy as np
    import torch

    from paper_2410_14088_amd import bmq
    from paper_2410_14088_amd import circuits as C

    inverse = None
    if args.workload == "qft":
        n = args.n or 30
        d = C.config(1, n=n)
        gates = d["gates"]
        fuse = args.fuse or 4
        wname = f"qft-on-ry-{n}q"
    elif args.workload == "random":
        n = args.n or 33
        d = C.config(2, n=n)
        gates = d["gates"]
        inverse = C.mirror(gates)[len(gates):]
        wname = f"random-u3-cz-{n}q-d16"
        fuse = args.fuse or 5
        if not args.fuse and not args.no_autotune:
            # tile size and fusion width by measurement (sv_autotune_space) on
            # the first four layers; Algorithm 1's inner size stays 2
            tune = autotune_headline(d, gates, args)
            fuse = tune["chosen"]["fuse_qubits"]
            args.tile = args.tile or tune["chosen"]["tile_qubits"]
    else:
        n = args.n or 33
        d = C.config(2, n=n)
        gates = C.mirror(d["gates"])
        fuse = args.fuse or 5
        wname = f"random-{n}q-d16-mirror"
    args.fuse = fuse
    d["domain"] = {"lin": 0, "log": 1, "raw": 2}[args.domain]
    d["eb"] = args.eb or d["eb"]
    cfg = bmq.Config(n=n, b=d["b"], inner=2, fuse=fuse, domain=d["domain"], eb=d["eb"], tile=args.tile,
                     flags=args.flags, pool_bytes=(64 << 20) if args.host_resident else 0)
    plan = bmq.Plan(gates, cfg)
    info = plan.info()
    G = len(gates)
    dev = "cuda:0"
    planning = None
    if args.workload == "random" and not args.no_predictor_pools and not args.host_resident:
        # device pools sized by the learned predictor's rollout of this plan
        planning = headline_pools(plan, n, d["b"], fuse, args.tile or 12, args.flags, d["eb"])
        cfg = bmq.Config(n=n, b=d["b"], inner=2, fuse=fuse, domain=d["domain"], eb=d["eb"], tile=args.tile,
                         flags=args.flags, pool_bytes=planning["pool_bytes"])
    sv = bmq.State(cfg, dev)
    if planning:
        # second memory level: records beyond the predicted device pools
        # spill to a pinned host pool instead of failing
        sv.attach_host_pool(planning["host_pool_bytes"])
    if args.host_resident:
        sv.attach_host_pool(2 * (8 << n))          # two state copies of up to complex64 size
    stream = torch.cuda.current_stream()

    def step(stats=True):
        sv.reset()
        return sv.apply(plan, stats=stats)

    progress(f"{wname}: {info['stages']} stages, {info['passes']} passes; warm-up")
    for _ in range(max(1, args.warmup) if planning else args.warmup):
        try:
            step()
        except bmq.BmqError as e:
            if not planning or e.code != -3:
                raise
            # the prediction fell short: worst-case pools (records are the same)
            progress("memory planning: predicted pools overflowed, worst-case pools")
            planning["fallback"] = True
            sv.close()
            torch.cuda.empty_cache()
            cfg = bmq.Config(n=n, b=d["b"], inner=2, fuse=fuse, domain=d["domain"], eb=d["eb"], tile=args.tile,
                             flags=args.flags)
            sv = bmq.State(cfg, dev)
            step()
    torch.cuda.synchronize()
    if planning:
        planning["warmup_host_spill_bytes"] = int(max(s["bytes_out_host"] for s in step()))
        if planning["warmup_host_spill_bytes"]:
            # the prediction fell short and records spilled to the host level:
            # time the headline with worst-case device pools (same records)
            progress("memory planning: records spilled to the host pool, worst-case pools for the timing")
            planning["fallback"] = True
            sv.close()
            torch.cuda.empty_cache()
            cfg = bmq.Config(n=n, b=d["b"], inner=2, fuse=fuse, domain=d["domain"], eb=d["eb"], tile=args.tile,
                             flags=args.flags)
            sv = bmq.State(cfg, dev)
            step()
        torch.cuda.synchronize()
    progress(f"{wname}: timing {args.steps} steps")

    all_stats = []
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(args.steps):
        all_stats.append(step())
    ev1.record(stream)
    torch.cuda.synchronize()
    total_ms = ev0.elapsed_time(ev1)
    ms_per_step = total_ms / args.steps
    progress(f"{wname}: {ms_per_step:.1f} ms per step")

    # algorithmic bytes and kernel time of the pass kernels over the timed
    # steps (HIP events the library records on its stream around each stage)
    alg_bytes = 0
    kern_ms = 0.0
    launches = 0
    for st in all_stats:
        for s in st:
            alg_bytes += s["bytes_in"] + s["bytes_out"] + s["dir_bytes"]
            kern_ms += s["ms"]
            launches += s["launches"]
    achieved = alg_bytes / (kern_ms * 1e-3) / 1e9
    last = all_stats[-1]
    peak_bytes = max(s["bytes_out"] for s in last)
    ratio64 = (8 << n) / peak_bytes
    ratio128 = (16 << n) / peak_bytes
    compressions = sum(s["passes"] for s in last) if args.flags & bmq.SV_FLAG_NO_SCRATCH else len(last)

    # result check outside the timed region
    peak_bytes_final = sv.footprint()[0]
    fwd = sv.fidelity_full(None)
    norm2 = fwd["norm2"]
    eps = 2.0 ** d["eb"] - 1 if d["domain"] == 1 else 0.0
    if args.workload == "qft":
        # sampled closed-form amplitudes
        rng = np.random.default_rng(1)
        idx = rng.integers(0, 1 << n, 4096).astype(np.uint64)
        want = qft_ry_closed_form(n, d["thetas"], idx)
        got = sv.amplitudes(torch.from_numpy(idx.astype(np.int64))).cpu().numpy().astype(np.complex128)
        f_est = float(abs(np.vdot(want, got)) ** 2 / (np.vdot(want, want).real * np.vdot(got, got).real))
        maxerr = float(np.abs(got - want).max())
        check = "4096 sampled amplitudes vs closed form"
        comp_total = compressions
    elif args.workload == "random":
        # the inverse circuit brings the exact state back to |0...0>: F^2 of
        # forward + inverse is |psi(0)|^2 / |psi|^2, exactly
        iplan = bmq.Plan(inverse, cfg)
        ist = sv.apply(iplan, stats=True)
        a0 = complex(sv.amplitudes(torch.zeros(1, dtype=torch.int64)).cpu().numpy()[0])
        f_est = abs(a0) ** 2 / sv.fidelity(None)[2]
        maxerr = abs(abs(a0) - 1.0)
        check = ("exact: after the timed forward steps the inverse circuit is applied and "
                 "F^2 = |psi(0)|^2 / |psi|^2 of forward + inverse")
        comp_total = compressions + len(ist)
    else:
        # the mirror circuit returns to |0...0>: F^2 = |psi(0)|^2 / |psi|^2 exactly
        a0 = complex(sv.amplitudes(torch.zeros(1, dtype=torch.int64)).cpu().numpy()[0])
        f_est = abs(a0) ** 2 / norm2
        maxerr = abs(abs(a0) - 1.0)
        check = "exact: mirror circuit, |psi(0)|^2 / |psi|^2"
        comp_total = compressions
    # rigorous lower bound: each compression moves the state by an angle of
    # at most arcsin(2^eb - 1) (LOG domain), and gates preserve angles
    bound = math.cos(min(math.pi / 2, comp_total * math.asin(eps))) ** 2 if eps else None

    prof_key = args.workload if (args.domain == "log" and args.eb in (0.0, 1e-5) and not args.host_resident) \
        else "other"
    arena = int(sv.arena.numel())
    scratch = 0 if args.flags & bmq.SV_FLAG_NO_SCRATCH else 8 << (
        min(n, max(d["b"] + 2, args.tile or 12)) if args.flags & bmq.SV_FLAG_GROUP_SCRATCH else n)
    out = {
        "metric": METRIC,
        "value": (2 ** n) * G / (ms_per_step * 1e-3),
        "unit": "amplitude·gates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": wname, "n_qubits": n, "block_qubits": d["b"], "gates": G,
                   "stages": info["stages"], "passes": info["passes"], "fused_ops": info["ops"],
                   "domain": args.domain, "eb": d["eb"], "fuse_qubits": args.fuse,
                   "tile_qubits": args.tile or 12, "flags": args.flags},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": counter_traffic(n, args.tile, args.fuse, args.flags, prof_key)},
        "alu_roofline": valu_profile(n, args.tile, args.fuse, args.flags, prof_key),
        "gbps_algorithmic": achieved,
        "kernel_ms_per_step": kern_ms / args.steps,
        "pass_launch_avg_ms": kern_ms / launches,
        "alg_bytes_per_launch": alg_bytes / launches,
        "pass_launches_per_step": launches // args.steps,
        "compression_ratio_vs_complex64": ratio64,
        "compression_ratio_vs_complex128": ratio128,
        "device_arena_bytes": arena,
        "device_scratch_bytes": scratch,
        "fidelity_f2": f_est,
        "fidelity_f2_bound": bound,
        "fidelity_check": check,
        "max_abs_err": maxerr,
        "norm2": norm2,
    }
    if planning:
        planning.setdefault("fallback", False)
        planning["actual_peak_record_bytes"] = int(peak_bytes)
        planning["timed_host_spill_bytes"] = int(sum(s["bytes_out_host"] for st in all_stats for s in st))
        out["device_arena_bytes"] = int(sv.arena.numel())
        out["memory_planning"] = planning
    if args.workload == "random" and not args.fuse_given and not args.no_autotune:
        out["autotune"] = tune
        out["config"]["fuse_qubits_autotuned"] = True
    if args.host_resident:
        out["config"]["host_resident"] = True
        out["host_share_of_records"] = sum(s["bytes_out_host"] for s in last) / max(1, sum(s["bytes_out"] for s in last))
    if args.persistent:
        # every stage in one queue launch; same records as the per-pass launches
        for _ in range(args.warmup):
            sv.reset()
            bmq.persistent_apply([sv], [plan])
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(args.steps):
            sv.reset()
            bmq.persistent_apply([sv], [plan])
        ev1.record(stream)
        torch.cuda.synchronize()
        out["persistent_ms_per_step"] = ev0.elapsed_time(ev1) / args.steps
        out["persistent_footprint_equal"] = sv.footprint()[0] == peak_bytes_final
    # a planner variant of Algorithm 1 on the same circuit and state, timed
    # the same way; the headline above stays on Algorithm 1 as written.  The
    # QFT gains from the diagonal-free rule (its phase ladders are diagonal),
    # random layers from commutation (a layer's gates commute).
    variant = {"qft": ("diagonal_free", bmq.SV_FLAG_DIAGONAL_FREE),
               "random": ("commute", bmq.SV_FLAG_COMMUTE),
               "random-mirror": ("commute", bmq.SV_FLAG_COMMUTE)}.get(args.workload)
    plan_flags = bmq.SV_FLAG_GATE_PER_STAGE | bmq.SV_FLAG_DIAGONAL_FREE | bmq.SV_FLAG_COMMUTE
    if variant and not args.flags & plan_flags and not args.host_resident and not args.no_variant:
        vname, vflag = variant
        vcfg = bmq.Config(n=n, b=d["b"], inner=2, fuse=fuse, domain=d["domain"], eb=d["eb"], tile=args.tile,
                          flags=args.flags | vflag)
        vplan = bmq.Plan(gates, vcfg)
        vinfo = vplan.info()
        vsteps = max(1, min(args.steps, args.variant_steps))
        sv.reset()
        sv.apply(vplan, stats=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(vsteps):
            sv.reset()
            sv.apply(vplan, stats=True)
        ev1.record(stream)
        torch.cuda.synchronize()
        vms = ev0.elapsed_time(ev1) / vsteps
        progress(f"planner variant {vname}: {vms:.1f} ms per step")
        res = {"value": (2 ** n) * G / (vms * 1e-3), "ms_per_step": vms, "steps": vsteps,
               "stages": vinfo["stages"], "passes": vinfo["passes"]}
        if args.workload == "qft":
            rng = np.random.default_rng(1)
            idx = rng.integers(0, 1 << n, 4096).astype(np.uint64)
            want = qft_ry_closed_form(n, d["thetas"], idx)
            got = sv.amplitudes(torch.from_numpy(idx.astype(np.int64))).cpu().numpy().astype(np.complex128)
            res["fidelity_f2"] = float(abs(np.vdot(want, got)) ** 2 / (np.vdot(want, want).real * np.vdot(got, got).real))
            res["max_abs_err_sampled"] = float(np.abs(got - want).max())
        elif args.workload == "random":
            icfg = bmq.Config(n=n, b=d["b"], inner=2, fuse=fuse, domain=d["domain"], eb=d["eb"], tile=args.tile,
                              flags=args.flags | vflag)
            sv.apply(bmq.Plan(inverse, icfg))
            a0 = complex(sv.amplitudes(torch.zeros(1, dtype=torch.int64)).cpu().numpy()[0])
            res["fidelity_f2"] = abs(a0) ** 2 / sv.fidelity(None)[2]
        else:
            a0 = complex(sv.amplitudes(torch.zeros(1, dtype=torch.int64)).cpu().numpy()[0])
            res["fidelity_f2"] = abs(a0) ** 2 / sv.fidelity(None)[2]
        out[vname] = res
    if args.workload in ("qft", "random") and not args.no_variant and not args.host_resident and \
            not args.flags & ~bmq.SV_FLAG_GROUP_SCRATCH:
        # qubit remapping (SV_FLAG_REMAP): swaps keep the soonest-used qubits
        # in the blocks; the state ends with its qubits at the plan's layout
        rcfg = bmq.Config(n=n, b=d["b"], inner=2, fuse=fuse, domain=d["domain"], eb=d["eb"], tile=args.tile,
                          flags=args.flags | bmq.SV_FLAG_REMAP)
        rplan = bmq.Plan(gates, rcfg)
        rsteps = max(1, min(args.steps, args.variant_steps))
        sv.reset()
        sv.apply(rplan)
        torch.cuda.synchronize()
        ev0.record(stream)
        for _ in range(rsteps):
            sv.reset()
            sv.apply(rplan)
        ev1.record(stream)
        torch.cuda.synchronize()
        rms = ev0.elapsed_time(ev1) / rsteps
        progress(f"planner variant remap: {rms:.1f} ms per step")
        res = {"value": (2 ** n) * G / (rms * 1e-3), "ms_per_step": rms, "steps": rsteps,
               "stages": rplan.n_stages, "passes": rplan.info()["passes"],
               "swaps": sum(1 for i in rplan.gate_order() if i == 0xFFFFFFFF) // 3}
        if args.workload == "qft":
            lay = rplan.layout()
            rng = np.random.default_rng(1)
            idx = rng.integers(0, 1 << n, 4096).astype(np.uint64)
            pidx = np.zeros_like(idx)
            for L, pos in enumerate(lay):
                pidx |= ((idx >> np.uint64(L)) & np.uint64(1)) << np.uint64(pos)
            want = qft_ry_closed_form(n, d["thetas"], idx)
            got = sv.amplitudes(torch.from_numpy(pidx.astype(np.int64))).cpu().numpy().astype(np.complex128)
            res["fidelity_f2"] = float(abs(np.vdot(want, got)) ** 2 / (np.vdot(want, want).real * np.vdot(got, got).real))
        else:
            # forward + inverse planned together returns to |0...0> whatever the layout
            mplan = bmq.Plan(C.mirror(gates), rcfg)
            sv.reset()
            sv.apply(mplan)
            a0 = complex(sv.amplitudes(torch.zeros(1, dtype=torch.int64)).cpu().numpy()[0])
            res["fidelity_f2"] = abs(a0) ** 2 / sv.fidelity(None)[2]
            res["fidelity_check"] = "forward + inverse planned together with remapping, |psi(0)|^2 / |psi|^2"
        out["remap"] = res
    if args.workload == "random" and not args.no_variant and not args.host_resident and \
            not args.flags & ~bmq.SV_FLAG_GROUP_SCRATCH:
        # the fusion comparison of the configuration: 5-qubit matrices on the
        # matrix cores against 1- and 2-qubit operations as vector
        # butterflies in LDS (whichever the headline is not)
        def timed(vcfg, vsteps):
            vplan = bmq.Plan(gates, vcfg)
            sv.reset()
            sv.apply(vplan)
            torch.cuda.synchronize()
            ev0.record(stream)
            for _ in range(vsteps):
                sv.reset()
                sv.apply(vplan)
            ev1.record(stream)
            torch.cuda.synchronize()
            vms = ev0.elapsed_time(ev1) / vsteps
            progress(f"variant fusion {vcfg.fuse}, inner {vcfg.inner}: {vms:.1f} ms per step")
            sv.apply(bmq.Plan(inverse, vcfg))
            a0 = complex(sv.amplitudes(torch.zeros(1, dtype=torch.int64)).cpu().numpy()[0])
            return {"value": (2 ** n) * G / (vms * 1e-3), "ms_per_step": vms, "steps": vsteps,
                    "fuse_qubits": vcfg.fuse, "inner_size": vcfg.inner, "tile_qubits": vcfg.tile or 12,
                    "stages": vplan.info()["stages"], "passes": vplan.info()["passes"],
                    "fidelity_f2": abs(a0) ** 2 / sv.fidelity(None)[2]}
        vsteps = max(1, min(args.steps, args.variant_steps))
        for name, k in (("mfma_5q", 5), ("lds_butterflies", 2)):
            if k != fuse:
                out[name] = timed(bmq.Config(n=n, b=d["b"], inner=2, fuse=k, domain=d["domain"], eb=d["eb"],
                                             tile=args.tile), vsteps)
        if not args.no_autotune:
            # Algorithm 1's inner size (the stage size) by measurement as well:
            # fewer, larger stages (fewer compressions), more passes per stage
            sv.close()
            sv = None
            torch.cuda.empty_cache()
            st_tune = autotune_headline(d, gates, args, inner=(2, 3, 4, 5), fuse=(fuse,),
                                        tiles=(args.tile or 12,))
            icfg = bmq.Config(n=n, b=d["b"], inner=st_tune["chosen"]["inner_size"], fuse=fuse, domain=d["domain"],
                              eb=d["eb"], tile=args.tile, flags=args.flags)
            sv = bmq.State(icfg, dev)
            out["autotuned_stage_size"] = dict(timed(icfg, vsteps), autotune=st_tune)
    if args.stats_out:
        with open(args.stats_out, "w") as f:
            json.dump(last, f, indent=1)
    if args.workload == "random" and not args.no_batch and not args.host_resident:
        # the batched workload (512 uneven circuits of 18-26 qubits) in the same run
        sv.close()
        sv = None
        torch.cuda.empty_cache()
        progress("batched workload: 512 circuits")
        b = batch_line(args)
        progress("batched workload done")
        out["batch"] = {k: b[k] for k in ("value", "ms_per_step", "config", "sequential_ms", "speedup_vs_sequential",
                                          "persistent_ms", "compression_ratio_vs_complex64", "planning")}
    if not args.no_cpu_baseline and args.workload in ("qft", "random"):
        if sv is not None:
            sv.close()
            sv = None
        torch.cuda.empty_cache()
        cn = args.cpu_n or 30
        out["cpu_baseline"] = cpu_baseline(args.workload, cn, args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
