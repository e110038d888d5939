#!/usr/bin/env python3
"""Throughput of the biasing-force path on one MI355X.

Workload (default): 256 walkers with atom counts log-uniform in [22, 5000]
and private hill lists of 1k-50k hills each (about 6.5M hills), two periodic
dihedral CVs per walker, well-tempered metadynamics (sigma 0.35 rad,
w 1.2 kJ/mol, bias factor 6, T 300 K, stride 500).  One step = CVs and their
Jacobian for every walker, the hill sum with dV/dxi, the force gather onto
the atoms (added to the force buffer) and the well-tempered deposition, for
all walkers; the steps are replayed from a captured HIP graph.

Printed: one JSON line with steps/s (value), hill evaluations per second,
the hill-sum kernel's bandwidth against the HBM roofline, and the FP64 CPU
oracle timed on a bounded sample of the same workload.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--graph-steps", type=int, default=50, help="steps per captured graph")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target length of the CPU sample")
    ap.add_argument("--hill-reps", type=int, default=200, help="launches timed for the hill-sum kernel")
    ap.add_argument("--probe-copy-mb", type=int, default=0,
                    help="after the run, copy this many MiB with the plain copy probe (counter calibration)")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the surrogate workload")
    ap.add_argument("--no-bust", action="store_true", help="skip the cache-busting replica of the hill kernel")
    ap.add_argument("--no-cn3", action="store_true", help="skip the cell-list coordination-number workload")
    ap.add_argument("--no-sweep", action="store_true", help="skip the one-walker hill-count sweep")
    ap.add_argument("--no-umbrella", action="store_true", help="skip the harmonic-window workload")
    ap.add_argument("--no-abf", action="store_true", help="skip the ABF workload")
    ap.add_argument("--no-wtmd22", action="store_true", help="skip the 22-atom 1,000-step workload")
    ap.add_argument("--cn3-steps", type=int, default=50, help="timed steps of the coordination-number workload")
    ap.add_argument("--tuning-cache", default=os.path.join(ROOT, "paper_2301_04835_amd", "tuning_mi355x.json"),
                    help="autotuner cache (JSON): an entry for this problem shape is reused, else searched and added")
    ap.add_argument("--sg-train-steps", type=int, default=100000, help="Adam steps of the surrogate fit")
    ap.add_argument("--sg-steps", type=int, default=2000, help="timed steps of each surrogate-workload path")
    return ap.parse_args()


def build_context(d, p):
    import torch
    from paper_2301_04835_amd import Sampler

    W = p["n_walkers"]
    s = Sampler(0)
    s.add_cvs(d["cvs"])
    s.set_walkers(d["atom_off"], d["n_hills"] + 64)
    s.metad(p["sigma"], p["w"], p["T"], p["bias_factor"], p["stride"], 1)
    s.bind()
    hoff = d["hill_off"]
    for w in range(W):
        s.hills_set(w, d["centers"][hoff[w]:hoff[w + 1]], d["heights"][hoff[w]:hoff[w + 1]])
    pos = torch.from_numpy(d["pos"]).cuda()
    forces = torch.zeros_like(pos)
    return s, pos, forces


TRAFFIC_SOURCES = ("k_bias.hip", "dev_cv.h", "dev_gather.h", "dev_reduce.h", "sx_api.cpp")  # kernels + state layout


def kernel_sources_sha():
    """sha256 (first 16 hex digits) of the tile kernel's sources and of the
    library source that lays out the state it reads."""
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_2301_04835_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(tile):
    """HBM bytes per launch of the tile kernel at this tile size, from the
    committed counter summary, or None if the kernel's sources changed since
    the counters were taken."""
    path = os.path.join(ROOT, "profiles", "hill_tiles_walkers256_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.strip().split("=", 1)
            kv[k.strip()] = v.strip()
    key = "traffic_bytes_per_launch.tile%d" % tile
    if kv.get("kernel_sources_sha") != kernel_sources_sha() or key not in kv:
        return None
    return float(kv[key])


def cpu_baseline(d, p, target_s):
    """The FP64 oracle on the host: whole steps (CVs, hill sums, chain rule)
    over all 256 walkers, single thread, repeated until ~target_s seconds;
    then the same with the hill sums spread over the host's cores (OpenMP,
    walkers in parallel; a third of the time)."""
    import oracle

    W = p["n_walkers"]
    off, hoff = d["atom_off"], d["hill_off"]
    C = d["centers"].astype(np.float64)
    H = d["heights"].astype(np.float64)
    per = [2 * np.pi, 2 * np.pi]

    def one_step(nthreads):
        xi = np.zeros((W, 2))
        Js = []
        for w in range(W):
            xi[w], J = oracle.cv_eval(d["pos"][off[w]:off[w] + 8].astype(np.float64), d["cvs"])
            Js.append(J)
        V, dV = oracle.hillsum_batch(xi, hoff, C, H, p["sigma"], per, nthreads=nthreads)
        for w in range(W):
            oracle.chain_rule(-dV[w], Js[w])

    def rate(nthreads, seconds):
        n = 0
        t0 = time.perf_counter()
        while True:
            one_step(nthreads)
            n += 1
            el = time.perf_counter() - t0
            if el >= seconds:
                return n, el

    n, el = rate(1, target_s)
    nt = host_cores()
    n_all, el_all = rate(nt, target_s / 3.0)
    return {"value": n / el, "unit": "steps/s", "cores": 1, "kind": "oracle",
            "sample": "%d full steps of the same 256-walker workload (%d hills per step), FP64, 1 thread, %.1f s"
                      % (n, int(hoff[-1]), el),
            "all_cores": {"value": n_all / el_all, "unit": "steps/s", "cores": nt,
                          "sample": "%d full steps, hill sums over %d OpenMP threads, %.1f s" % (n_all, nt, el_all)}}


def host_cores():
    """Threads the host gives this process: the CPU affinity set, capped by
    OMP_NUM_THREADS when that is set."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    env = os.environ.get("OMP_NUM_THREADS", "")
    return max(1, min(n, int(env))) if env.isdigit() else n


def bust_leg(d, p, tile, grid, reps):
    """The hill-sum kernel on four copies of the workload at once (1,024
    walkers, about 310 MB of hills: above the 256 MB Infinity Cache, so no
    launch finds its hills in the cache of the previous one); the same tiling.
    Returns the kernel's algorithmic read rate, i.e. an HBM-only figure."""
    import torch
    from paper_2301_04835_amd import Sampler

    R, W = 4, p["n_walkers"]
    na = int(d["atom_off"][-1])
    atom_off = np.concatenate([d["atom_off"][:-1] + r * na for r in range(R)] + [[R * na]])
    s = Sampler(0)
    s.add_cvs(d["cvs"])
    s.set_walkers(atom_off, np.tile(d["n_hills"] + 64, R))
    s.metad(p["sigma"], p["w"], p["T"], p["bias_factor"], p["stride"], 1)
    s.bind()
    hoff = d["hill_off"]
    for r in range(R):
        for w in range(W):
            s.hills_set(r * W + w, d["centers"][hoff[w]:hoff[w + 1]], d["heights"][hoff[w]:hoff[w + 1]])
    s.set_tuning(tile, grid)
    pos = torch.from_numpy(np.tile(d["pos"], (R, 1))).cuda()
    forces = torch.zeros_like(pos)
    ms_a, ms_b = s.time_hill(pos, forces=forces, reps=reps)
    nbytes = int(np.sum(s.hill_counts())) * 12
    return {"walkers": R * W, "hill_bytes": nbytes, "kernel_ms": ms_a, "finalize_kernel_ms": ms_b,
            "achieved": nbytes / (ms_a * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": nbytes / (ms_a * 1e-3) / 1e9 / HBM_PEAK_GBS}


def graph_len(steps, cap):
    """Steps per captured graph: the largest divisor of `steps` that is at
    most `cap`, so that exactly `steps` steps are timed in whole graphs."""
    for g in range(max(1, min(cap, steps)), 0, -1):
        if steps % g == 0:
            return g
    return 1


def stream_probe(nbytes, reps=200):
    """The plain streaming-read probe (non-temporal float4 loads, the hill
    kernel's kind) over the same number of bytes, 2,048 workgroups: the
    practical ceiling of a read-bound kernel of this size, in GB/s."""
    import ctypes
    import torch
    from paper_2301_04835_amd import _lib

    M = _lib.load_measure()
    nb = nbytes // 16 * 16
    src = torch.ones(nb // 4, device="cuda")
    sink = torch.zeros(2048, device="cuda")
    st = torch.cuda.current_stream()
    call = lambda: M.sx_probe_read(ctypes.c_void_p(src.data_ptr()), nb, ctypes.c_void_p(sink.data_ptr()), 2048, 1,
                                   ctypes.c_void_p(st.cuda_stream))
    for _ in range(10):
        call()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        call()
    e1.record(st)
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    return {"bytes": nb, "us": us, "achieved": nb / us / 1e3, "unit": "GB/s", "loads": "non-temporal float4"}


def capacity_leg(d, p, tile, grid, reps, factor=4):
    """The 256-walker hill-sum kernel with each walker's capacity reserved at
    `factor` x its hill count (as a run that preallocates for the hills it
    will deposit): the kernel's time follows the hills present, not the
    space reserved."""
    import torch
    from paper_2301_04835_amd import Sampler

    s = Sampler(0)
    s.add_cvs(d["cvs"])
    s.set_walkers(d["atom_off"], factor * d["n_hills"])
    s.metad(p["sigma"], p["w"], p["T"], p["bias_factor"], p["stride"], 1)
    s.bind()
    hoff = d["hill_off"]
    for w in range(p["n_walkers"]):
        s.hills_set(w, d["centers"][hoff[w]:hoff[w + 1]], d["heights"][hoff[w]:hoff[w + 1]])
    s.set_tuning(tile, grid)
    pos = torch.from_numpy(d["pos"]).cuda()
    forces = torch.zeros_like(pos)
    ms_a, ms_b = s.time_hill(pos, forces=forces, reps=reps)
    nbytes = int(np.sum(s.hill_counts())) * 12
    return {"capacity_over_count": factor, "capacity_hills": int(factor * d["n_hills"].sum()),
            "hills": int(np.sum(s.hill_counts())), "kernel_ms": ms_a, "finalize_kernel_ms": ms_b,
            "achieved": nbytes / (ms_a * 1e-3) / 1e9, "unit": "GB/s"}


def wtmd22_leg(args):
    """The 22-atom workload: phi/psi of one chain, 2,000 hills whose heights
    follow the well-tempered law (deposited one after another on the GPU),
    sigma 0.35 rad, w 1.2 kJ/mol, bias factor 6, T 300 K, stride 500; 1,000
    steps with fresh FP64 positions each step (template + N(0, 0.02^2) nm),
    one library call per step as an engine makes it, returning xi, V,
    dV/dxi and the atom forces of every step."""
    import torch
    from paper_2301_04835_amd import Sampler, synth

    p = synth.WTMD22
    d = synth.wtmd22_inputs()
    s = Sampler(0)
    s.add_cvs(d["cvs"])
    s.metad(list(p["sigma"]), p["w"], p["T"], p["bias_factor"], p["stride"], p["n_hills"] + 8)
    s.bind()
    xs = torch.from_numpy(d["centers"].astype(np.float64)).cuda()
    for k in range(p["n_hills"]):  # the well-tempered sequence: each hill sees the ones before it
        s.deposit(xs[k:k + 1])
    T = p["n_steps"]
    frames = torch.from_numpy(d["frames"]).cuda()
    F = torch.zeros((T, p["n_atoms"], 3), dtype=torch.float32, device="cuda")
    xi = torch.zeros((T, 1, 2), dtype=torch.float64, device="cuda")
    V = torch.zeros((T, 1), dtype=torch.float64, device="cuda")
    dV = torch.zeros((T, 1, 2), dtype=torch.float64, device="cuda")
    for t in range(20):  # warm-up on a scratch force buffer, no deposition
        s.step(frames[t], forces=F[0], step=1, V_out=V[0])
    F.zero_()
    # each step's buffers as views made before the clock starts: the slicing
    # is the harness's bookkeeping, not the library's work
    bufs = [(frames[t], F[t], xi[t], V[t], dV[t]) for t in range(T)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for t, (x, f, o1, o2, o3) in enumerate(bufs):
        s.step(x, forces=f, step=t, xi_out=o1, V_out=o2, dV_out=o3)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    s.check()
    return {"workload": "wtmd22-2000-hills-1000-steps", "atoms": p["n_atoms"], "hills": p["n_hills"],
            "steps": T, "steps_per_s": T / el, "ms_per_step": el * 1e3 / T,
            "calls": "one sx_step per step (fresh positions), eager", "hills_after": int(s.hill_counts()[0])}


def wtmd22_oracle(d_unused=None):
    """CPU oracle leg of the 22-atom workload: its 1,000 steps (CVs, hill sum
    over 2,000 well-tempered hills, chain rule, deposits at steps 0 and 500),
    FP64, one thread."""
    import oracle
    from paper_2301_04835_amd import synth

    p = synth.WTMD22
    d = synth.wtmd22_inputs()
    kdT = oracle.KB * (p["bias_factor"] - 1.0) * p["T"]
    C = d["centers"].astype(np.float64)
    H = oracle.wt_sequence(C, p["w"], kdT, p["sigma"], [2 * np.pi, 2 * np.pi], round_f32=True)
    C, H = list(C), list(H)
    t0 = time.perf_counter()
    for t in range(d["frames"].shape[0]):
        o = oracle.metad_step(d["frames"][t], d["cvs"], np.array(C), np.array(H), p["sigma"], p["w"], kdT,
                              p["stride"], t)
        if o["deposit"] is not None:
            C.append(o["deposit"][0])
            H.append(o["deposit"][1])
    el = time.perf_counter() - t0
    return {"value": d["frames"].shape[0] / el, "unit": "steps/s", "cores": 1, "kind": "oracle",
            "sample": "all %d steps, FP64, 1 thread, %.2f s" % (d["frames"].shape[0], el)}


def timed_graph(s, pos, forces, outs, steps, warmup, gsteps=10, sys_forces=None):
    """Capture gsteps steps in a HIP graph, replay warmup, then time
    replays for `steps` steps (wall clock around synchronisations)."""
    import torch
    xi, V, dV = outs
    s.graph_capture(gsteps, pos, forces=forces, xi_out=xi, V_out=V, dV_out=dV, sys_forces=sys_forces)
    for _ in range(max(1, warmup // gsteps)):
        s.graph_launch()
    torch.cuda.synchronize()
    n = max(1, steps // gsteps)
    t0 = time.perf_counter()
    for _ in range(n):
        s.graph_launch()
    torch.cuda.synchronize()
    return n * gsteps / (time.perf_counter() - t0), n * gsteps


def sweep_leg(reps):
    """One walker of the 22-atom system (phi/psi dihedrals) with K = 2^11 ...
    2^26 private hills (24 KB ... 805 MB): the hill kernel's algorithmic read
    rate as the list grows from cache-resident past the 256 MB Infinity
    Cache.  Tile 4096, one workgroup per tile; the CVs are fused."""
    import torch
    from paper_2301_04835_amd import Sampler, synth

    p = synth.WTMD22
    Ks = [1 << e for e in (11, 14, 17, 20, 23, 26)]
    C = synth.uniform_centers(Ks[-1], 2, 7)
    H = synth.uniform_heights(Ks[-1], 8)
    pos = torch.from_numpy(synth.chain_template(p["n_atoms"], 1).astype(np.float32)).cuda()
    forces = torch.zeros_like(pos)
    rows = []
    for K in Ks:
        s = Sampler(0)
        s.add_cvs(synth.backbone_cvs(4))
        s.set_walkers(np.array([0, p["n_atoms"]]), [K + 64])
        s.metad(list(p["sigma"]), p["w"], p["T"], p["bias_factor"], p["stride"], K + 64)
        s.bind()
        s.hills_set(0, C[:K], H[:K])
        s.set_tuning(4096, 0)
        ms_a, ms_b = s.time_hill(pos, forces=forces, reps=reps if K < (1 << 23) else max(10, reps // 10))
        gbs = 12.0 * K / (ms_a * 1e-3) / 1e9
        rows.append({"hills": K, "hill_bytes": 12 * K, "kernel_ms": ms_a, "finalize_kernel_ms": ms_b,
                     "hill_evals_per_s": K / (ms_a * 1e-3), "achieved": gbs, "frac": gbs / HBM_PEAK_GBS})
        del s
        torch.cuda.empty_cache()
    return {"workload": "wtmd22-one-walker-hill-sweep", "unit": "GB/s", "peak": HBM_PEAK_GBS, "rows": rows}


def umbrella_leg(args, d):
    """Harmonic biasing with one window per walker on the 256-walker
    workload (uneven walkers, the same two dihedrals): window centres along
    a path across the (phi, psi) torus, k = 100 kJ/mol/rad^2; replayed
    graphs of whole steps (CVs, spring, forces, window sums), then umbrella
    integration of the windows on the host."""
    import torch
    from paper_2301_04835_amd import Sampler

    W = len(d["atom_off"]) - 1
    t = np.linspace(0.0, 1.0, W)
    centers = np.stack([-2.5 + 5.0 * t, 1.5 - 3.0 * t], 1)
    s = Sampler(0)
    s.add_cvs(d["cvs"])
    s.set_walkers(d["atom_off"])
    s.harmonic([100.0, 100.0], centers)
    s.bind()
    pos = torch.from_numpy(d["pos"]).cuda()
    forces = torch.zeros_like(pos)
    mk = lambda *sh: torch.zeros(sh, dtype=torch.float64, device="cuda")
    rate, nst = timed_graph(s, pos, forces, (mk(W, 2), mk(W), mk(W, 2)), args.steps, args.warmup)
    s.check()
    t0 = time.perf_counter()
    _, A = s.umbrella_integrate()
    t_int = time.perf_counter() - t0
    return {"workload": "umbrella-windows-256-walkers", "walkers": W, "k": [100.0, 100.0],
            "steps_per_s": rate, "ms_per_step": 1e3 / rate, "steps_timed": nst,
            "integrate_s": t_int, "A_range": float(np.max(A) - np.min(A))}


def abf_leg(args):
    """ABF on (Rg of 500 atoms, coordination number between two groups of
    1,000 atoms, all pairs, rational switch r0 = 0.5 nm, 6/12) in a
    50,000-atom box of 10 nm, 100 x 100 bins, threshold 500: two eager steps,
    the second kept for the oracle check, then 10^4 steps in replayed graphs.
    Positions and system forces (N(0, 100^2) kJ/mol/nm) stay fixed, so every
    sample lands in one bin, which must then hold exactly one count per step."""
    import torch
    from paper_2301_04835_amd import Sampler, synth

    p = synth.ABF50K
    cvs = synth.abf50k_cvs()
    box = [p["box"]] * 3
    s = Sampler(0)
    s.add_cvs(cvs)
    s.set_box(box)
    s.set_walkers(np.array([0, p["n_atoms"]]))
    s.abf(list(p["lo"]), list(p["hi"]), list(p["nbins"]), p["n_threshold"])
    s.bind()
    pos_np = synth.abf50k_box(seed=2)
    fs_np = np.random.default_rng(12).normal(0.0, p["fsys_sd"], size=pos_np.shape).astype(np.float32)
    pos, fs = torch.from_numpy(pos_np).cuda(), torch.from_numpy(fs_np).cuda()
    forces = torch.zeros_like(pos)
    mk = lambda *sh: torch.zeros(sh, dtype=torch.float64, device="cuda")
    out = (mk(1, 2), mk(1), mk(1, 2))
    for t in range(2):  # the second step carries the first sample's bias
        forces.zero_()
        s.step(pos, forces=forces, xi_out=out[0], V_out=out[1], dV_out=out[2], sys_forces=fs)
    first = (out[0].cpu().numpy()[0], -out[2].cpu().numpy()[0], forces.cpu().numpy())
    warm = 200
    rate, nst = timed_graph(s, pos, forces, out, p["n_steps"], warm, gsteps=args.graph_steps, sys_forces=fs)
    s.check()
    N, _ = s.abf_grid(0)
    nsamp = 2 + (max(1, warm // args.graph_steps) + nst // args.graph_steps) * args.graph_steps
    res = {"workload": "abf-rg500-cn1000x1000-50k-atoms", "atoms": p["n_atoms"], "bins": list(p["nbins"]),
           "pairs_per_step": p["n_a"] * p["n_b"], "steps_per_s": rate, "ms_per_step": 1e3 / rate,
           "steps_timed": nst, "graph_steps": args.graph_steps,
           "samples_one_bin": bool(int(N.sum()) == nsamp and int((N > 0).sum()) == 1)}
    return res, (cvs, box, pos_np, fs_np, first)


def abf_oracle_check(ad):
    """CPU oracle leg of the ABF workload: the two eager steps recomputed in
    FP64 from the same inputs; the second step's CVs, bias along the CVs and
    atom forces are compared."""
    import oracle

    cvs, box, pos_np, fs_np, (xi, b, F) = ad
    from paper_2301_04835_amd import synth

    p = synth.ABF50K
    g = oracle.AbfGrid(list(p["lo"]), list(p["hi"]), list(p["nbins"]), [False, False], p["n_threshold"])
    fs = fs_np.astype(np.float64)
    t0 = time.perf_counter()
    x, J = oracle.cv_eval(pos_np.astype(np.float64), cvs, np.array(box))
    oracle.abf_step(g, x, J, fs)
    t_or = time.perf_counter() - t0  # one whole oracle step
    br, Fb, _, _ = oracle.abf_step(g, x, J, fs)
    rel = lambda a, r: float(np.max(np.abs(a - r)) / max(np.max(np.abs(r)), 1e-300))
    return {"oracle_step_s": t_or, "xi_rel_err_vs_oracle": [float(abs(xi[d] - x[d]) / abs(x[d])) for d in range(2)],
            "b_rel_err_vs_oracle": rel(b, br), "force_rel_err_vs_oracle": rel(F, Fb)}


def surrogate_leg(args):
    """Surrogate workload: 100,000 shared hills of a converged well-tempered
    run on two dihedral CVs (sigma 0.3 rad, w ~ U[0.5, 1.5] kJ/mol, T 300 K,
    bias factor 6); 256 walkers of 22 atoms; a 4-64-64-1 tanh network
    trained on the GPU on 2^17 torus points, certified on a 512^2 grid at
    0.1 kJ/mol/rad.  Exact path: the shared hill sum for every walker.
    Surrogate path: the network for every walker plus the exact sum for the
    walkers outside certified cells.  Both run as replayed graphs of whole
    steps (CVs, bias, forces); the bias is frozen (no deposition)."""
    import torch
    from paper_2301_04835_amd import Sampler, synth, synth_wt

    K, W = 100000, 256
    t0 = time.perf_counter()
    C, H = synth_wt.wt_hills(K)
    pos_np, off = synth.chain_walkers(W, 22, seed=4)
    t_gen = time.perf_counter() - t0
    s = Sampler(0)
    s.add_cvs(synth.backbone_cvs(4))
    s.set_walkers(off, [K], shared=True)
    s.metad([0.3, 0.3], 1.0, 300.0, 6.0, 0, K)
    s.surrogate(64, max_samples=1 << 17, max_batch=4096, cert_n=512, tol_force=0.1)
    s.bind()
    s.hills_set(0, C, H)
    g = np.random.default_rng(7)
    P0 = []
    for fan_in, shape in [(4, (64, 4)), (1, (64,)), (64, (64, 64)), (1, (64,)), (64, (64,)), (1, (1,))]:
        P0.append((g.uniform(-1, 1, shape) / np.sqrt(fan_in) if fan_in > 1 else np.zeros(shape)).ravel())
    s.surrogate_params(np.concatenate(P0).astype(np.float32))
    X = torch.from_numpy(synth_wt.torus_points(1 << 17, 8)).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss = s.surrogate_train(X, batch=4096, steps=args.sg_train_steps, lr=3e-3, lr_final=1e-5)
    t_train = time.perf_counter() - t0
    t0 = time.perf_counter()
    frac = s.surrogate_certify()
    t_cert = time.perf_counter() - t0
    pos = torch.from_numpy(pos_np).cuda()
    forces = torch.zeros_like(pos)
    mk = lambda *sh: torch.zeros(sh, dtype=torch.float64, device="cuda")
    ex = (mk(W, 2), mk(W), mk(W, 2))
    sg = (mk(W, 2), mk(W), mk(W, 2))
    rate_exact, n_ex = timed_graph(s, pos, forces, ex, args.sg_steps, 200)
    s.surrogate_enable(True)
    rate_sg, n_sg = timed_graph(s, pos, forces, sg, args.sg_steps, 200)
    nfb = s.surrogate_fallback_count()
    s.check()
    dv_net = sg[2].cpu().numpy()
    dv_ex = ex[2].cpu().numpy()
    err_vs_exact = float(np.max(np.linalg.norm(dv_net - dv_ex, axis=1)))
    res = {"workload": "wtmd-surrogate-100k-shared-256-walkers", "hills": K, "walkers": W,
           "network": "4-64-64-1 tanh, bf16 weights, FP32 accumulate", "train_steps": args.sg_train_steps,
           "train_batch": 4096, "train_samples": 1 << 17, "train_loss": loss, "train_s": t_train,
           "certify_grid": "512x512", "certify_s": t_cert, "certified_fraction": frac,
           "fallback_walkers": nfb, "exact_steps_per_s": rate_exact, "surrogate_steps_per_s": rate_sg,
           "speedup": rate_sg / rate_exact, "steps_timed": n_sg,
           "max_dV_err_vs_exact_gpu": err_vs_exact, "tol_force": 0.1, "input_gen_s": t_gen}
    return res, (C, H, pos_np, off, sg)


def grid_leg(args, sg_data, exact_rate, n=512):
    """The surrogate workload's bias kept on an n x n grid (multilinear
    read-back of V and dV/dxi; the 100,000 hills summed once onto the nodes):
    replayed graphs of whole steps, bias frozen as in the surrogate leg.  The
    read-back's force error against the exact hill sum (GPU, FP64 sums) at
    2^14 random torus points and at the walkers."""
    import torch
    from paper_2301_04835_amd import Sampler, synth, synth_wt

    C, H, pos_np, off, _ = sg_data
    K, W = len(H), len(off) - 1
    s = Sampler(0)
    s.add_cvs(synth.backbone_cvs(4))
    s.set_walkers(off, [K + 64], shared=True)
    s.metad([0.3, 0.3], 1.0, 300.0, 6.0, 0, K + 64)
    s.metad_grid([-np.pi, -np.pi], [np.pi, np.pi], [n, n])
    s.bind()
    t0 = time.perf_counter()
    s.hills_set(0, C, H)  # fills the grid (synchronous)
    t_build = time.perf_counter() - t0
    pos = torch.from_numpy(pos_np).cuda()
    forces = torch.zeros_like(pos)
    mk = lambda *sh: torch.zeros(sh, dtype=torch.float64, device="cuda")
    out = (mk(W, 2), mk(W), mk(W, 2))
    rate, nst = timed_graph(s, pos, forces, out, args.sg_steps, 200)
    s.check()
    X = torch.from_numpy(synth_wt.torus_points(1 << 14, 9)).cuda()
    _, Gg = s.grid_eval(X)
    _, Ge = s.bias_eval(X)
    e = torch.linalg.norm(Gg - Ge, dim=1)
    _, Gw = s.bias_eval(out[0])
    ew = torch.linalg.norm(out[2] - Gw, dim=1)
    res = {"grid": "%d x %d nodes, multilinear read-back" % (n, n), "grid_fill_s": t_build,
           "steps_per_s": rate, "steps_timed": nst, "speedup_vs_exact": rate / exact_rate,
           "max_dV_err_vs_exact_random_points": float(e.max()), "rms_dV_err_vs_exact_random_points":
           float(torch.sqrt((e ** 2).mean())), "max_dV_err_vs_exact_gpu_walkers": float(ew.max())}
    return res, (C, H, out[0].cpu().numpy(), out[2].cpu().numpy())


def grid_oracle_check(gd):
    """CPU oracle leg of the grid workload: the FP64 hill sum at the walkers'
    CV values, against which the grid step's dV/dxi error is stated."""
    import oracle

    C, H, xi, dv = gd
    _, dVr = oracle.hillsum_batch(xi, None, C.astype(np.float64), H.astype(np.float64), [0.3, 0.3],
                                  [2 * np.pi, 2 * np.pi], nthreads=1)
    err = np.linalg.norm(dv - dVr, axis=1)
    return {"max_dV_err_vs_oracle": float(err.max()), "median_dV_err_vs_oracle": float(np.median(err))}


FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X FP32 vector (packed) peak


def rho_cand(p):
    """Candidate partners per home atom of the cell-list pair pass: the
    partner group's density times the 3 x 3 x (2 rz + 1) sub-cells around the
    home sub-cell (rz = 4 z sub-cells per cut length, 10 cells per edge)."""
    nc = int(np.floor(p["box"] / p["rcut"]))
    clen = p["box"] / nc
    return p["n_group"] / p["box"] ** 3 * (3 * clen) ** 2 * (9 * clen / 4)


def cn3_leg(args):
    """512 walkers, each 60,000 atoms uniform in a 12 nm periodic box; three
    coordination numbers between 20,000-atom groups (r0 0.5 nm, (6, 12), hard
    cut 1.2 nm, divided by |A|) through cell lists; one shared list of 10^6
    three-dimensional hills (sigma 0.2) around the expected CN.  One step =
    cell sort, one pair pass (CN values and each member's gradients), hill
    sum, forces gathered from the stored gradients (VJP); replayed graphs.
    Then the same with a 6-128-128-1 surrogate."""
    import torch
    from paper_2301_04835_amd import Sampler, synth

    p = synth.CN3
    W, n, K = 512, p["n_group"], 1000000
    cvs = synth.cn3_cvs(n, p["r0"], p["rcut"])
    pos_np, off = synth.cn3_positions(W, n, p["box"])
    C, H = synth.cn3_hills(K, mean=p["cn_mean"], sd=p["hill_sd"])
    s = Sampler(0)
    s.add_cvs(cvs)
    s.set_box([p["box"]] * 3)
    s.set_walkers(off, [K + 64 * W], shared=True)
    s.metad([p["sigma"]] * 3, 1.0, 300.0, 6.0, 0, K + 64 * W)
    s.surrogate(128, max_samples=1 << 17, max_batch=2048, cert_n=48, tol_force=1.0)
    s.bind()
    s.hills_set(0, C, H)
    pos = torch.from_numpy(pos_np).cuda()
    forces = torch.zeros_like(pos)
    mk = lambda *sh: torch.zeros(sh, dtype=torch.float64, device="cuda")
    ex = (mk(W, 3), mk(W), mk(W, 3))
    rate, nst = timed_graph(s, pos, forces, ex, args.cn3_steps, 10, gsteps=5)
    ms_sort, ms_pairs, ms_vjp = s.time_cell(pos, forces=forces, reps=10)
    # algorithmic work: expected pairs inside the cut (density x sphere volume);
    # the pair pass evaluates each from both sides (each side: r^2 8 flops,
    # switch and its derivative 9, switch sum 1, 3 FMAs 6).  The cells make it
    # visit 9 x 2.25 cut-length cubes per atom, 4.8x the cut sphere: the
    # candidate rate is reported beside it
    cand = 2 * 3 * W * n * rho_cand(p)
    rho = n / p["box"] ** 3
    pairs = 3 * W * n * rho * 4.0 / 3.0 * np.pi * p["rcut"] ** 3
    pass_flops = 2 * pairs * 24
    res = {"workload": "cn3-cells-512-walkers-1M-shared-hills", "walkers": W, "atoms_per_walker": 3 * n,
           "cvs": "CN_AB, CN_BC, CN_CA over 20,000-atom groups, cut 1.2 nm",
           "cells": "10 x 10 x 40 (z cut into 4 sub-cells per cut length)", "hills": K,
           "steps_per_s": rate, "ms_per_step": 1e3 / rate, "steps_timed": nst,
           "cell_sort_ms": ms_sort, "pair_pass_ms": ms_pairs, "vjp_gather_ms": ms_vjp,
           "pairs_in_cut_per_step": pairs, "candidate_pairs_per_step": cand,
           "candidate_pairs_per_s": cand / (ms_pairs * 1e-3),
           "roofline": {"bound": "alu", "kernel": "k_cell_jac<true> (+ k_cn_cell_fin)",
                        "achieved": pass_flops / (ms_pairs * 1e-3) / 1e12, "peak": FP32_VECTOR_PEAK_TFLOPS,
                        "unit": "TFLOP/s", "frac": pass_flops / (ms_pairs * 1e-3) / 1e12 / FP32_VECTOR_PEAK_TFLOPS,
                        "flops_per_launch": pass_flops, "traffic": None}}
    # surrogate: 6-128-128-1 on standardised CNs, certified on a 48^3 grid
    # over mean +- 1.2; tolerance 1e-3 of the rms gradient of the bias (the
    # bias of 10^6 hills reaches ~10^5 kJ/mol: an absolute tolerance of the
    # dihedral workloads' size has no meaning here)
    g = np.random.default_rng(12)
    X = torch.from_numpy(p["cn_mean"] + p["hill_sd"] * g.normal(size=(1 << 17, 3))).cuda()
    s.surrogate_norm([p["cn_mean"]] * 3, [p["hill_sd"]] * 3)
    P0 = []
    for fan_in, shape in [(6, (128, 6)), (1, (128,)), (128, (128, 128)), (1, (128,)), (128, (128,)), (1, (1,))]:
        P0.append((g.uniform(-1, 1, shape) / np.sqrt(fan_in) if fan_in > 1 else np.zeros(shape)).ravel())
    s.surrogate_params(np.concatenate(P0).astype(np.float32))
    t0 = time.perf_counter()
    s.surrogate_train(X, batch=2048, steps=20000, lr=3e-3, lr_final=1e-5)
    t_train = time.perf_counter() - t0
    Vx, dVx = s.bias_eval(X[:4096])
    g_rms = float(torch.sqrt((dVx ** 2).sum(1).mean()).item())
    lo, hi = [p["cn_mean"] - 1.2] * 3, [p["cn_mean"] + 1.2] * 3
    tol = 1e-3 * g_rms
    s.surrogate_tolerance(tol)
    frac = s.surrogate_certify(lo, hi)
    s.surrogate_enable(True)
    sg = (mk(W, 3), mk(W), mk(W, 3))
    rate_sg, _ = timed_graph(s, pos, forces, sg, args.cn3_steps, 10, gsteps=5)
    nfb = s.surrogate_fallback_count()
    s.surrogate_enable(False)
    res["surrogate"] = {"network": "6-128-128-1 tanh on (u, u^2), bf16 weights", "train_steps": 20000,
                        "train_s": t_train, "certify_grid": "48^3 over mean +- 1.2", "tol_force": tol,
                        "rms_bias_gradient": g_rms, "certified_fraction": frac, "fallback_walkers": nfb,
                        "steps_per_s": rate_sg, "speedup": rate_sg / rate}
    return res, (pos_np, off, cvs, p)


def cn3_oracle(cn_data):
    """CPU oracle leg: one walker's three coordination numbers and their
    gradients (brute force over all pairs, FP64, one thread)."""
    import oracle

    pos_np, off, cvs, p = cn_data
    t0 = time.perf_counter()
    oracle.cv_eval(pos_np[off[0]:off[1]].astype(np.float64), cvs, np.full(3, p["box"]))
    el = time.perf_counter() - t0
    return {"oracle_s_per_walker_cvs_and_gradients_1_thread": el}


def surrogate_oracle_check(sg_data):
    """CPU oracle leg of the surrogate workload: the FP64 hill sum at the
    walkers' CV values, against which the surrogate step's dV/dxi error is
    stated (timed as the oracle's cost of one exact step's bias)."""
    import oracle

    C, H, pos_np, off, sg = sg_data
    xi = sg[0].cpu().numpy()
    dv = sg[2].cpu().numpy()
    t0 = time.perf_counter()
    _, dVr = oracle.hillsum_batch(xi, None, C.astype(np.float64), H.astype(np.float64), [0.3, 0.3],
                                  [2 * np.pi, 2 * np.pi], nthreads=1)
    el = time.perf_counter() - t0
    err = np.linalg.norm(dv - dVr, axis=1)
    return {"max_dV_err_vs_oracle": float(err.max()), "median_dV_err_vs_oracle": float(np.median(err)),
            "oracle_bias_s_per_step_1_thread": el}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: the batched-walker path runs on a single MI355X; "
              "multi-GPU sharding is a design note only (--gpus %d not supported)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_2301_04835_amd import synth

    p = synth.WALKERS256
    d = synth.walkers_inputs(n_walkers=p["n_walkers"], seed=3)
    K_total = int(d["hill_off"][-1])
    s, pos, forces = build_context(d, p)
    W = p["n_walkers"]
    xi = torch.zeros((W, 2), dtype=torch.float64, device="cuda")
    V = torch.zeros(W, dtype=torch.float64, device="cuda")
    dV = torch.zeros((W, 2), dtype=torch.float64, device="cuda")
    # first eager step (also provides xi for tuning), then tile autotune
    s.step(pos, forces=forces, xi_out=xi, V_out=V, dV_out=dV)
    torch.cuda.synchronize()
    s.autotune(pos, cache_path=args.tuning_cache)
    tile, grid = s.get_tuning()
    gsteps = graph_len(args.steps, args.graph_steps)
    s.graph_capture(gsteps, pos, forces=forces, xi_out=xi, V_out=V, dV_out=dV)
    for _ in range(max(1, args.warmup // gsteps)):
        s.graph_launch()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    nlaunch = args.steps // gsteps
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(nlaunch):
        s.graph_launch()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    steps = nlaunch * gsteps
    s.check()
    ms_step = wall * 1e3 / steps
    ev_ms_step = e0.elapsed_time(e1) / steps
    # hill counts after the run (deposits every `stride` steps add hills)
    counts_total = int(np.sum(s.hill_counts()))
    # the step's hill-sum kernels alone: hipEvents around back-to-back
    # launches on the context's stream (same configuration as the step;
    # no deposition), tile kernel (A) and finalize kernel (B) separately
    ms_a, ms_b = s.time_hill(pos, forces=forces, reps=args.hill_reps)
    # the two as a step runs them, and what a launch in a graph costs alone
    ms_pair, ms_noop = s.time_hill_step(pos, forces=forces, reps=args.hill_reps)
    bytes_per_launch = counts_total * 12  # 2 float32 centres + 1 float32 height per hill
    achieved = bytes_per_launch / (ms_a * 1e-3) / 1e9
    traffic = measured_traffic(tile)
    out = {
        "metric": "biased steps/s (CV+bias+force), 256 walkers",
        "value": steps / wall,
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "event_ms_per_step": ev_ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (FP64 sums)",
        "data": "synthetic",
        "config": {"workload": "wtmd-walkers-256", "walkers": W, "hills_total": counts_total,
                   "atoms_total": int(d["atom_off"][-1]), "cvs": "2 dihedrals per walker", "sigma": p["sigma"],
                   "tile_hills": tile, "grid": grid, "graph_steps": gsteps},
        "hill_evals_per_s": counts_total * steps / wall,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_hill_tiles%s<2,%d,fused,float>" % ("_persist" if grid else "", tile // 1024),
                     "kernel_ms": ms_a,
                     "finalize_kernel_ms": ms_b, "pair_ms": ms_pair, "noop_launch_ms": ms_noop,
                     "bytes_per_launch": bytes_per_launch},
    }
    if args.probe_copy_mb:
        import ctypes
        from paper_2301_04835_amd import _lib
        M = _lib.load_measure()
        nb = args.probe_copy_mb << 20
        src = torch.ones(nb // 4, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            M.sx_probe_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), nb, 2048,
                            ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
        torch.cuda.synchronize()
    out["stream_probe"] = stream_probe(bytes_per_launch)
    out["capacity_4x_count"] = capacity_leg(d, p, tile, grid, args.hill_reps)
    if not args.no_wtmd22:
        out["wtmd22"] = wtmd22_leg(args)
    if not args.no_bust:
        out["roofline_above_infinity_cache"] = bust_leg(d, p, tile, grid, args.hill_reps)
    if not args.no_sweep:
        out["hill_sweep_one_walker"] = sweep_leg(args.hill_reps)
    if not args.no_umbrella:
        out["umbrella"] = umbrella_leg(args, d)
    ad = None
    if not args.no_abf:
        out["abf"], ad = abf_leg(args)
    sg_data = gd = None
    if not args.no_surrogate:
        out["surrogate"], sg_data = surrogate_leg(args)
        out["surrogate"]["bias_grid"], gd = grid_leg(args, sg_data, out["surrogate"]["exact_steps_per_s"])
    cn_data = None
    if not args.no_cn3:
        out["cn3"], cn_data = cn3_leg(args)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(d, p, args.cpu_seconds)
        if sg_data is not None:
            out["surrogate"].update(surrogate_oracle_check(sg_data))
            out["surrogate"]["bias_grid"].update(grid_oracle_check(gd))
        if cn_data is not None:
            out["cn3"].update(cn3_oracle(cn_data))
        if ad is not None:
            out["abf"].update(abf_oracle_check(ad))
        if "wtmd22" in out:
            out["wtmd22"]["cpu_oracle"] = wtmd22_oracle()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
