"""Benchmark of the Brownian hard-disk time step on one MI355X.

A "step" is one full pass of the hot path: all-pairs force, Euler-Maruyama
update with noise, device flip repair of the Delaunay triangulation and the
overlap-correction rounds (each with its repair).  Default workload: N=65,536
disks, all-pairs inverse-square force in FP32, two species with a
non-reciprocal strength matrix, self-propulsion v0=1, Dr=1, area fraction 0.40
(synthetic random-sequential-insertion positions).

Prints one JSON line.  `value` is particle-steps/s with all state resident in
HBM; `roofline` reports the all-pairs force kernel (the dominant kernel)
against the FP32 vector ALU peak using 12 flops per ordered pair, from HIP
events recorded on the library's stream around each force launch;
`cpu_baseline` times the sequential FP64 oracle for one full step of the same
workload on one host core.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particle-steps/s (N=65,536 all-pairs; N=1M Verlet); % of VALU/HBM roofline"
FLOPS_PER_PAIR = 12            # 2 sub, 3 for d^2, 1 rsqrt, 2 mul for d^-3, 2 FMAs (2 flops each)
PEAK_FP32_TFLOPS = 157.3       # MI355X published FP32 vector peak (packed FMA)
PEAK_FP32_NONPACKED = 78.6     # 256 CU x 64 lanes x 2 flops x 2.4 GHz without packed FP32
PEAK_FP64_TFLOPS = 78.6

# HBM bytes per k_force launch on the default workload from two rocprofv3 --pmc passes
# (FETCH_SIZE, WRITE_SIZE), each scaled by the same counter's reading for a plain
# 1 GiB copy; valid only for the force kernel's source it was measured on (sha1 of
# the force section of k_particles.hip, see force_source_sha1).
MEASURED_TRAFFIC = {"sha1": "6bb720c9c1b32473e48c7b3a46cc513746b3524c", "workload": "C2", "n": 65536,
                    "force_config": {"chunk": 1024, "per_lane": 4, "persistent": 2},
                    "bytes_per_launch": 2.0 * 2205.0 * 1024 + 1.0 * 32768.0 * 1024}


FORCE_KERNELS = {0: "k_force", 1: "k_force_queue", 2: "k_force_sym"}
# VALU instructions per pair evaluation in the force kernels' inner loops (read off their gfx950 ISA):
# ordinary forms, per ordered pair: 2 sub, mul + FMA for d^2, v_rsq, 2 mul for d^-3, 2 FMA;
# symmetric form (FP32), per unordered pair: the same, 2 FMA for j's side, and one DPP move
# (a step moves x, y and both sums of each of a lane's 2 j: 8 moves for its 8 pairs)
VALU_PER_PAIR = {0: 9.0, 1: 9.0}   # symmetric form: 11 + 4 / per_lane (the 4 moves per j are shared by per_lane i)
LANE_ISSUE_PER_S = 256 * 4 * 16 * 2.4e9   # CUs x SIMDs x lanes x clock: one VALU lane-op per slot


def valu_issue_frac(fcfg, n, seconds, fp32):
    """Fraction of the VALU issue slots the force launch used (FP32 only; FP64 math is not one op per flop)."""
    if not fp32:
        return None
    form = fcfg["persistent"]
    pairs = n * (n - 1) / 2 if form == 2 else n * (n - 1)
    per_pair = 11.0 + 4.0 / fcfg["per_lane"] if form == 2 else VALU_PER_PAIR[form]
    return per_pair * pairs / seconds / LANE_ISSUE_PER_S


def force_source_sha1():
    """sha1 of the all-pairs force section of k_particles.hip (d^-3, pair loops, tiles, launches)."""
    import hashlib

    src = os.path.join(ROOT, "paper_1703_02484_amd", "csrc", "k_particles.hip")
    with open(src) as fh:
        text = fh.read()
    a = text.index("// ---------------------------------------------------------------- forces")
    b = text.index("// F_i = sum_c K[s_i][spec(c)] Phi_{i,c} over the chunks")
    return hashlib.sha1(text[a:b].encode()).hexdigest()


def measured_traffic(workload, n, fcfg):
    h = force_source_sha1()
    m = MEASURED_TRAFFIC
    if h != m["sha1"] or workload != m["workload"] or n != m["n"]:
        return None
    if any(fcfg[k] != v for k, v in m["force_config"].items()):   # counted on another launch configuration
        return None
    return m["bytes_per_launch"]


# HBM bytes per dispatch of the short-range step's full passes (N = 1,048,576, the C3 workload) from two
# rocprofv3 --pmc passes (FETCH_SIZE x 2, WRITE_SIZE x 1, calibrated on a plain copy), beside the algorithmic
# bytes; valid for the kernel sources they were counted on (sha1 of the three kernel files, see
# c3_source_sha1).  MB = 1e6 bytes.
C3_TRAFFIC = {"sha1": "a3d772a99d6da0544405237dc6d1be9af153ea52", "kernels": {
    "k_flip_eval_full": {"measured_MB": 100.2, "algorithmic_MB": 84.1},
    "k_ovl_detect": {"measured_MB": 72.0, "algorithmic_MB": 67.4},
    "k_em": {"measured_MB": 101.0, "algorithmic_MB": 100.7},
    "k_force_nl": {"measured_MB": 61.9, "algorithmic_MB": 54.5},
    "k_skin_check": {"measured_MB": 33.6, "algorithmic_MB": 33.6},
    "k_snapshot": {"measured_MB": 109.6, "algorithmic_MB": 109.6}}}


def c3_source_sha1():
    """sha1 of the kernel sources of the short-range step's full passes."""
    import hashlib

    h = hashlib.sha1()
    for f in ("k_topology.hip", "k_verlet.hip", "k_particles.hip"):
        with open(os.path.join(ROOT, "paper_1703_02484_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _short_range_once(w, steps, warmup, overlap):
    import torch

    from paper_1703_02484_amd import binding

    sim = binding.Sim.from_workload(w, overlap=overlap)
    sim.set_graph_mode(True)
    sim.step(warmup)
    st0 = sim.state()[3]
    sim.enable_kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()   # every stream of the device, the library's included
    elapsed = time.perf_counter() - t0
    force_ms, launches = sim.kernel_time()
    st1 = sim.state()[3]
    sim.close()
    d = {k: st1[k] - st0[k] for k in st1}
    return elapsed, force_ms / 1e3 / max(launches, 1), d


def run_short_range(steps, warmup):
    """Secondary measurement: the short-range workload (N = 1,048,576, phi = 0.5, FP32 list force), with the
    overlap rounds over Delaunay edges (the library's default) and over the neighbour lists (the paper's
    short-range algorithm, Sec. 5, no triangulation)."""
    from paper_1703_02484_amd import synth

    w = synth.make("C3")
    # algorithmic bytes of k_force_nl per disk: own position 16, count 4, ~4 list entries x 4 (mean
    # neighbours within cutoff + skin at phi = 0.5), force 16 (neighbour positions come from cache)
    bytes_per_disk = 16 + 4 + 4 * 4 + 16
    out = {"workload": f"C3: N={w.n} screened A=1 lam=0.5 cutoff 2.5 skin 0.5, Verlet lists, "
                       f"{'FP32' if w.fp32_forces else 'FP64'} pair forces, phi=0.50, dt={w.dt}"}
    for overlap in ("delaunay", "verlet"):
        elapsed, avg_s, d = _short_range_once(w, steps, warmup, overlap)
        gbs = bytes_per_disk * w.n / avg_s / 1e9
        rounds = d["overlap_rounds_total"] / steps
        if overlap == "delaunay":
            # algorithmic bytes per disk: update 96 (it also writes the (x, y) pairs), force, one repair scan
            # 64, first overlap detection 64, per overlap round gather + apply 84, list rebuild amortised 10
            step_bytes = w.n * (96 + bytes_per_disk + 64 + 64 + 84 * rounds + 10)
        else:
            # update 96, force, per detection (rounds + 1) a full list pass 40, per round apply 16 per moved
            # disk (counted as the full pass's share), list rebuild amortised 10
            step_bytes = w.n * (96 + bytes_per_disk + 40 * (rounds + 1) + 10)
        step_gbs = step_bytes * steps / elapsed / 1e9
        out[overlap] = {
            "value": w.n * steps / elapsed, "unit": "particle-steps/s", "steps": steps, "warmup": warmup,
            "ms_per_step": 1e3 * elapsed / steps, "overlap_method": overlap,
            "force_nl_ms": avg_s * 1e3, "force_nl_gbs_algorithmic": gbs, "force_nl_frac_hbm": gbs / 8000.0,
            "step_gbs_algorithmic": step_gbs, "step_frac_hbm": step_gbs / 8000.0,
            "overlap_rounds_per_step": rounds, "overlap_pairs_per_step": d["overlap_edges_total"] / steps,
            "flips_per_step": d["flips_total"] / steps, "verlet_rebuilds": d["verlet_rebuilds"],
            "kinetic_repairs": d["kinetic_repairs"], "host_rebuilds": d["host_rebuilds"],
            "host_continued_steps": d["host_continued"]}
    out["traffic_per_dispatch"] = C3_TRAFFIC["kernels"] if C3_TRAFFIC["sha1"] == c3_source_sha1() else None
    # headline of this secondary line: the library's default (Delaunay overlap correction)
    out.update({k: out["delaunay"][k] for k in ("value", "unit", "steps", "warmup", "ms_per_step")})
    return out


def loop_pin(cfg):
    """bd_params options that give a single-system handle the batch's force form: same chunking, particles
    per lane and launch form, so each system's sums are cut and added in the same order."""
    if cfg["persistent"] == 2:
        return {"force_chunk": {4: -1, 2: -2, 8: -3}[cfg["per_lane"]]}
    return {"force_chunk": cfg["chunk"], "force_per_lane": cfg["per_lane"], "force_launch": cfg["persistent"]}


def run_batched(steps, warmup, loop_steps):
    """Batched systems (256 replicas, N_r log-uniform in [2048, 32768], FP64) in one handle, against a loop
    that steps one handle per system pinned to the batch's own force form (same chunks, same launch form,
    same summation order).  After timing, every single handle is advanced to the batch's step and its
    positions are compared with its system in the batch (equal accuracy means identical positions)."""
    import numpy as np
    import torch

    from paper_1703_02484_amd import binding, synth

    ws = synth.make_batch(256)
    ntot = sum(w.n for w in ws)
    pairs = sum(w.n * (w.n - 1) for w in ws)
    b = binding.Sim.from_workloads(ws)
    b.set_graph_mode(True)
    cfg = b.force_config()
    b.step(warmup)
    st0 = b.state()[3]
    b.enable_kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    force_ms, launches = b.kernel_time()
    xb, _, step_b, st1 = b.state()
    _, doff, _ = b.layout()
    b.close()
    avg_s = force_ms / 1e3 / max(launches, 1)
    tflops = FLOPS_PER_PAIR * pairs / avg_s / 1e12
    out = {"workload": f"C4: {len(ws)} systems, N_r log-uniform in [2048, 32768] (sum {ntot}), phi_r ~ U[0.2, 0.5], "
                       f"FP64 all-pairs inverse-square K=1e-2, dt=1e-4, seed_r=r",
           "value": ntot * steps / elapsed, "unit": "particle-steps/s", "steps": steps, "warmup": warmup,
           "ms_per_step": 1e3 * elapsed / steps, "pair_interactions_per_s": pairs / avg_s,
           "force_ms": avg_s * 1e3, "force_tflops": tflops, "force_frac_fp64": tflops / PEAK_FP64_TFLOPS,
           "force_config": cfg,
           "overlap_rounds_per_step": (st1["overlap_rounds_total"] - st0["overlap_rounds_total"]) / steps,
           "host_rebuilds": st1["host_rebuilds"], "host_continued_steps": st1["host_continued"]}
    # the same batch with FP32 pair sums (positions and predicates stay FP64)
    b32 = binding.Sim.from_workloads(ws, fp32=True)
    b32.set_graph_mode(True)
    b32.step(warmup)
    b32.enable_kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b32.step(steps)
    torch.cuda.synchronize()
    el32 = time.perf_counter() - t0
    f32_ms, f32_launches = b32.kernel_time()
    out["fp32"] = {"value": ntot * steps / el32, "unit": "particle-steps/s", "ms_per_step": 1e3 * el32 / steps,
                   "force_ms": f32_ms / max(f32_launches, 1),
                   "force_tflops": FLOPS_PER_PAIR * pairs / (f32_ms / 1e3 / max(f32_launches, 1)) / 1e12,
                   "force_config": b32.force_config()}
    b32.close()
    # the same systems, one handle each (pinned to the batch's force form), stepped one after another
    pin = loop_pin(cfg)
    singles = [binding.Sim.from_workload(w, **pin) for w in ws]
    same_form = all(all(s.force_config()[k] == cfg[k] for k in ("chunk", "per_lane", "persistent"))
                    for s in singles)
    for s in singles:
        s.set_graph_mode(True)
        s.step(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(loop_steps):
        for s in singles:
            s.step(1)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # advance every single handle to the batch's step and compare positions
    worst = 0.0
    for r, s in enumerate(singles):
        s.step(step_b - 1 - loop_steps)
        worst = max(worst, float(np.abs(s.state()[0] - xb[doff[r]:doff[r + 1]]).max()))
        s.close()
    if worst != 0.0:
        print(f"warning: batch and per-system loop differ by {worst:.3e}", file=sys.stderr)
    out["per_system_loop"] = {"value": ntot * loop_steps / el, "unit": "particle-steps/s", "steps": loop_steps,
                              "ms_per_step": 1e3 * el / loop_steps, "force_pin": pin,
                              "same_force_form_as_batch": same_form,
                              "max_abs_position_diff_vs_batch": worst, "compared_at_step": step_b}
    out["speedup_vs_loop"] = out["value"] / out["per_system_loop"]["value"]
    return out


def run_ablation(steps):
    """j-broadcast ablation of the all-pairs force on the default workload (N = 65,536, FP32): the same tiles
    (chunks of 1024, 4 particles i per lane) with j as wave-uniform scalar loads or staged through LDS (the
    shared-memory broadcast of the paper's n-body kernel, Sec. 6), and the symmetric form that turns j
    around the wavefront by DPP.  Force launches timed with HIP events on the library's stream."""
    import numpy as np
    import torch

    from paper_1703_02484_amd import binding, synth

    w = synth.make("C2")
    pairs = w.n * (w.n - 1)
    forms = {"scalar_loads": dict(force_chunk=1024, force_per_lane=4, force_launch=0),
             "lds_staged": dict(force_chunk=1024, force_per_lane=4, force_launch=2),
             "dpp_symmetric": dict(force_chunk=-1)}
    out = {"workload": f"C2: N={w.n}, FP32 all-pairs inverse-square force", "steps": steps}
    forces = {}
    for name, pin in forms.items():
        sim = binding.Sim.from_workload(w, **pin)
        forces[name] = sim.forces()
        sim.set_graph_mode(True)
        sim.step(2)
        sim.enable_kernel_timing(True)
        sim.step(steps)
        torch.cuda.synchronize()
        ms, launches = sim.kernel_time()
        avg = ms / max(launches, 1)
        out[name] = {"force_ms": avg, "pair_interactions_per_s": pairs / (avg / 1e3),
                     "tflops_12_flop_convention": FLOPS_PER_PAIR * pairs / (avg / 1e3) / 1e12,
                     "force_config": sim.force_config()}
        sim.close()
    out["lds_vs_scalar_max_abs_force_diff"] = float(np.abs(forces["lds_staged"] - forces["scalar_loads"]).max())
    out["lds_over_scalar_time"] = out["lds_staged"]["force_ms"] / out["scalar_loads"]["force_ms"]
    out["scalar_over_dpp_time"] = out["scalar_loads"]["force_ms"] / out["dpp_symmetric"]["force_ms"]
    return out


def run_adjoint():
    """Gradient of the species-0 mean squared displacement after 50 steps (N = 16,384, FP64, contact factor 1/2)
    with respect to K and the initial positions: forward with checkpoints every 10 steps, then the adjoint sweep."""
    import numpy as np
    import torch

    from paper_1703_02484_amd import binding, synth

    w = synth.make("C5")
    warm = binding.Sim.from_workload(w)
    warm.adjoint_begin(10, 10)
    warm.adjoint_backward(np.zeros((w.n, 2)))
    warm.close()
    plain = binding.Sim.from_workload(w)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plain.step(50)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    plain.close()
    g = binding.Sim.from_workload(w)
    t0 = time.perf_counter()
    g.adjoint_begin(50, 10)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    xT = g.state()[0]
    s0 = w.species == 0
    lamT = np.zeros_like(xT)
    lamT[s0] = 2.0 * (xT[s0] - w.xy[s0]) / s0.sum()
    t0 = time.perf_counter()
    g.adjoint_backward(lamT)
    t_bwd = time.perf_counter() - t0
    st = g.state()[3]
    g.close()
    pairs = w.n * (w.n - 1)
    return {"workload": f"C5: N={w.n}, S=2, K=1e-2, FP64 all pairs, contact factor 1/2 (the contact option of the "
                        f"overlap rule; the paper's own runs use factor 1), 50 steps, checkpoints every 10, "
                        f"loss = MSD of species 0",
            "forward_plain_s": t_plain, "forward_with_checkpoints_s": t_fwd, "backward_s": t_bwd,
            "backward_over_forward": t_bwd / t_plain,
            "backward_pair_interactions_per_s": 2 * 50 * pairs / t_bwd,
            "adjoint_flops_per_pair": 28, "overlap_rounds_forward": st["overlap_rounds_total"]}


def _progress(msg):
    """One line per finished or started part, on stderr (the JSON line stays alone on stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_cpu():
    """Model name of the host CPU and the logical CPUs this process may use."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for ln in fh:
                if ln.startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return model, os.cpu_count(), usable


def cpu_baseline(w):
    import oracle

    o = oracle.OracleSim.from_workload(w)
    t0 = time.perf_counter()
    o.step(1)
    dt = time.perf_counter() - t0
    model, ncpu, usable = host_cpu()
    return {"value": w.n / dt, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "cpu_model": model, "nproc": ncpu, "usable_cpus": usable,
            "sample": f"1 full step of the same workload (N={w.n}), FP64 sequential oracle on one thread, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="C2")
    ap.add_argument("--n", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true", help="launch kernel by kernel instead of replaying graphs")
    ap.add_argument("--tail-mode", type=int, default=-1, choices=[-1, 0, 1, 2],
                    help="overlap rounds: 0 one launch per phase, 1 one workgroup, 2 large phases launched and the "
                         "rest in one workgroup, -1 automatic")
    ap.add_argument("--no-short-range", action="store_true", help="skip the secondary N=1M Verlet measurement")
    ap.add_argument("--no-batched", action="store_true", help="skip the secondary 256-system batched measurement")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the secondary gradient measurement")
    ap.add_argument("--no-ablation", action="store_true", help="skip the j-broadcast ablation of the force")
    ap.add_argument("--only", choices=["short_range", "batched", "adjoint", "ablation"], default=None,
                    help="run one secondary measurement alone and print its JSON (for profiling)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain device copy of known size (scale for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); multi-GPU sharding is a design note, "
              f"not implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1703_02484_amd import binding, synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    if args.copy_calibration:
        nbytes = 1 << 30
        a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration": {"bytes_read_per_dispatch": nbytes, "bytes_written_per_dispatch": nbytes,
                                               "dispatches": 5}}), flush=True)
        return
    if args.only:
        fn = {"short_range": lambda: run_short_range(max(10, args.steps // 4), 20),
              "batched": lambda: run_batched(max(5, args.steps // 20), 2, max(2, args.steps // 100)),
              "adjoint": run_adjoint,
              "ablation": lambda: run_ablation(max(5, args.steps // 20))}[args.only]
        print(json.dumps({args.only: fn()}), flush=True)
        return
    w = synth.make(args.workload, n=args.n)
    sim = binding.Sim.from_workload(w)
    sim.set_tail_mode(args.tail_mode)
    # the same steps launched kernel by kernel, for comparison with the graph replay timed below
    sim.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(max(1, args.steps // 4))
    torch.cuda.synchronize()
    eager_ms = 1e3 * (time.perf_counter() - t0) / max(1, args.steps // 4)
    sim.set_graph_mode(not args.no_graph)
    sim.step(args.warmup)
    st0 = sim.state()[3]
    sim.enable_kernel_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()   # every stream of the device, the library's included
    elapsed = time.perf_counter() - t0
    force_ms, launches = sim.kernel_time()
    st1 = sim.state()[3]
    fcfg = sim.force_config()

    n = w.n
    ms_per_step = 1e3 * elapsed / args.steps
    value = n * args.steps / elapsed
    pairs = n * (n - 1)
    avg_force_s = force_ms / 1e3 / max(launches, 1)
    achieved = FLOPS_PER_PAIR * pairs / avg_force_s / 1e12
    peak = PEAK_FP32_TFLOPS if w.fp32_forces else PEAK_FP64_TFLOPS
    d = {k: st1[k] - st0[k] for k in st1}
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 forces, f64 positions/predicates" if w.fp32_forces else "f64",
        "data": "synthetic (random sequential insertion, seeded)",
        "config": {
            "workload": f"{w.name}: N={n} all-pairs inverse-square force, {'FP32' if w.fp32_forces else 'FP64'} "
                        f"forces, S={w.S}, v0={w.v0}, Dr={w.Dr}, phi={n * np.pi / w.L ** 2:.2f}, dt={w.dt}, "
                        f"hard walls, Delaunay overlap correction",
            "N": n,
            "pair_interactions_per_s": pairs / avg_force_s,
            "force_ms_per_step": force_ms / max(launches, 1),
            "other_ms_per_step": ms_per_step - force_ms / max(launches, 1),
            "graph_mode": not args.no_graph,
            "eager_ms_per_step": eager_ms,
            "overlap_rounds_per_step": d["overlap_rounds_total"] / args.steps,
            "flips_per_step": d["flips_total"] / args.steps,
            "flip_rounds_per_step": d["flip_rounds_total"] / args.steps,
            "kinetic_repairs": d["kinetic_repairs"],
            "host_rebuilds": d["host_rebuilds"],
            "host_continued_steps": d["host_continued"],
        },
        "roofline": {
            "kernel": "all-pairs force (" + FORCE_KERNELS[fcfg["persistent"]] + ")",
            "force_config": fcfg,
            "flop_convention": "12 flops per ordered pair (the all-pairs force's work, however it is evaluated)",
            "valu_issue_frac": valu_issue_frac(fcfg, n, avg_force_s, w.fp32_forces),
            "bound": "alu",
            "achieved": achieved,
            "peak": peak,
            "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": measured_traffic(w.name, n, fcfg),
            "traffic_unit": "bytes per launch",
            "flops_per_launch": FLOPS_PER_PAIR * pairs,
            "avg_launch_ms": avg_force_s * 1e3,
            "launches": launches,
            "peak_nonpacked_fp32": PEAK_FP32_NONPACKED if w.fp32_forces else None,
            "frac_of_nonpacked": achieved / PEAK_FP32_NONPACKED if w.fp32_forces else None,
        },
    }
    _progress(f"main workload done: {ms_per_step:.3f} ms/step")
    if not args.no_short_range and args.workload == "C2":
        _progress("short-range workload")
        out["short_range"] = run_short_range(max(10, args.steps // 4), 20)
    if not args.no_batched and args.workload == "C2":
        _progress("batched workload")
        out["batched"] = run_batched(max(5, args.steps // 20), 2, max(2, args.steps // 100))
    if not args.no_adjoint and args.workload == "C2":
        _progress("adjoint workload")
        out["adjoint"] = run_adjoint()
    if not args.no_ablation and args.workload == "C2":
        _progress("force ablation")
        out["ablation"] = run_ablation(max(5, args.steps // 20))
    if not args.no_cpu_baseline:
        _progress("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
