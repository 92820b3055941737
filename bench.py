#!/usr/bin/env python3
"""Benchmark of the blocked SA-AMG solve phase on one MI355X.

Workload: Q1 hexahedral linear elasticity on the unit cube with 128^3 elements
(6,440,067 dofs, 3x3 blocks), per-element E ~ lognormal(0, 1) and nu ~ U[0.2, 0.35]
(material seed 11, redraw seed 1011), right-hand side U[-1, 1] (seed 12), x = 0 face
clamped; 4-level smoothed-aggregation hierarchy (3x3 fine, 3x6 / 6x6 prolongators,
6x6 coarse operators), Chebyshev(2)/point-block-Jacobi V-cycle inside CG to a
relative residual of 1e-8.

One step = one pass of the hot path on fresh operator values: blocked COO assembly of
the fine operator, Galerkin recompute A_c = P^T A P on every level (fixed patterns,
reused prolongators), smoother refresh (block-diagonal inverses, Lanczos estimates,
coarsest Cholesky), and the PCG solve.  Values alternate between two material draws,
so every step really recomputes.  Hierarchies timed: "fp64" (everything in FP64, the
paper's arithmetic) and the mixed variants (V-cycle hierarchy in FP32 with FP32
accumulation, optionally BF16 prolongators, the learned eigenbound or device
aggregation; FP64 PCG, fine residual SpMV and coarsest Cholesky).  The reported value
is PCG solve seconds + PtAP recompute seconds of the FP64 hierarchy (median over the
timed steps); the mixed figures and their speed-up are reported beside it.

Also reported: the HBM roofline of the fine 3x3 FP64 SpMV (bsr_spmv) measured with
HIP events, the Galerkin recompute's algorithmic bandwidth (ptap_roofline), and the
CPU oracle measured on this host on the 64^3 problem (one core, in a child process
while the GPU sections run), with the GPU's own time on that problem beside it.  The
last stdout line is the compact result; per-step records and the side sections (the
learned eigenbound at 96^3, a batch of 24 instances with 8 right-hand sides, the
triquadratic (Q2, 27-node) problem at 64^3 elements, finite-element assembly) go to
stderr as one "[bench] detail" JSON line and, with --detail-out, to a file.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "PCG solve s + PtAP recompute s at 128^3 elasticity; %HBM peak; mixed vs FP64"

# HBM traffic of the roofline kernel (fine 3x3 FP64 SpMV with symmetric reads at 128^3)
# from rocprofv3 FETCH_SIZE / WRITE_SIZE passes, scaled by the copy-kernel calibration;
# valid only for the kernel sources it was measured on (their SHA-256 below), else
# reported as null.  Summary and commands: profiles/bsr_spmv_fine_f64_128cube.md.
TRAFFIC_RECORD = {
    "sources_sha256": "892a7e82017996abe7144defdae117382aaddce8e76006c65a23a7a555f27c00",
    "fetch_bytes": 3458992128,   # FETCH_SIZE 1,688,961 KiB x 2.00 (copy calibration)
    "write_bytes": 53366784,     # WRITE_SIZE 52,116 KiB x 1.00
}
TRAFFIC_SOURCES = ("paper_2606_24748_amd/csrc/spmv_core.hpp", "paper_2606_24748_amd/csrc/bsr.hip",
                   "paper_2606_24748_amd/csrc/common.hpp")

# HBM traffic of one Galerkin recompute over all levels (FP64 hierarchy at 128^3: the
# six pair-list passes), from the same kind of counter passes; null once its sources
# change.  Summary: profiles/ptap_counters_128cube.md.
PTAP_TRAFFIC_RECORD = {
    "sources_sha256": "ad6696f0fa84ed15d7f74fa1396c3ee4378b199e4a69acbec0839a739ff6b56a",
    "fetch_bytes": 34558126080,  # FETCH_SIZE 16,874,085 KiB x 2.00
    "write_bytes": 5251006464,   # WRITE_SIZE 5,127,936 KiB x 1.00
}
PTAP_TRAFFIC_SOURCES = ("paper_2606_24748_amd/csrc/ptap.hip", "paper_2606_24748_amd/csrc/ptap_plan.hpp",
                        "paper_2606_24748_amd/csrc/ptap_symbolic.hip", "paper_2606_24748_amd/csrc/common.hpp")


def kernel_sources_sha256(sources=TRAFFIC_SOURCES) -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in sources:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(rec=TRAFFIC_RECORD, sources=TRAFFIC_SOURCES):
    if not rec or rec.get("sources_sha256") != kernel_sources_sha256(sources):
        return None
    return rec["fetch_bytes"] + rec["write_bytes"]


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse_args(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=128, help="elements per cube edge")
    ap.add_argument("--variants", default="mixed,mixed-mlp,mixed-bf16,mixed-luby,fp64",
                    help="comma list of mixed, mixed-mlp, mixed-bf16, mixed-luby, fp64")
    ap.add_argument("--probe-reps", type=int, default=30)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--probe-only", action="store_true",
                    help="only assemble the fine operator and run the SpMV probe and the copy calibration")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-solve section")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned-eigenbound section")
    ap.add_argument("--no-q2", action="store_true", help="skip the triquadratic (Q2) section")
    ap.add_argument("--q2-n", type=int, default=64, help="elements per edge of the Q2 problem")
    ap.add_argument("--no-fe", action="store_true", help="skip the finite-element assembly section")
    ap.add_argument("--fe-n", type=int, default=128, help="elements per edge of the FE assembly problem")
    ap.add_argument("--fe-scalar-n", type=int, default=64,
                    help="elements per edge of the blocked vs scalar COO comparison")
    ap.add_argument("--only-section", choices=("learned", "batch", "q2", "fe", "ptap"), default=None,
                    help="run only that section and print its result (profiling runs)")
    ap.add_argument("--learned-n", type=int, default=96, help="edge of the learned-eigenbound deployment problem")
    ap.add_argument("--learned-setups", type=int, default=3,
                    help="cold setups timed per learned-section variant (the median is reported)")
    ap.add_argument("--model", default=None, help="eigenbound model JSON (default: the packaged one)")
    ap.add_argument("--batch-eager", action="store_true",
                    help="also time the batched CG launched eagerly (no graph replay)")
    ap.add_argument("--cpu-baseline-only", action="store_true", help=argparse.SUPPRESS)
    ap.add_argument("--cpu-n", type=int, default=CPU_N, help="elements per edge of the oracle's CPU baseline problem")
    ap.add_argument("--no-config-s", action="store_true", help="skip the 64^3 FP64 section (the CPU baseline's problem)")
    ap.add_argument("--detail-out", default=None,
                    help="also write the full result (per-step records, side sections) to this JSON file")
    return ap.parse_args(argv)


# ----------------------------------------------------------------------------------
# CPU baseline: the oracle, one core, on the 64^3 problem (run in a child process that
# works while the GPU sections run)
# ----------------------------------------------------------------------------------
CPU_N = 64               # Q1 elasticity at 64^3 elements (823,875 dofs), 4-level hierarchy
CPU_SEEDS = (1, 1001, 2)  # materials, redrawn materials, right-hand side


def cpu_baseline_child(n: int) -> dict:
    """The oracle's hot path on one core: cold setup on the first material draw
    (untimed), then, on the redrawn materials, the Galerkin recompute over all levels
    and the PCG solve to 1e-8 with the V-cycle of the recomputed hierarchy (timed)."""
    try:
        cpus = sorted(os.sched_getaffinity(0))
        os.sched_setaffinity(0, {cpus[-1]})
    except (AttributeError, OSError):
        pass
    import numpy as np

    import synth
    from oracle import solve
    from oracle import sparse as S

    s0, s1, sb = CPU_SEEDS
    m = synth.make_mesh(n)
    i, j = synth.coo_indices(m)
    v0 = synth.coo_values(m, *synth.lame(*synth.materials(m.n_elem, s0)))
    v1 = synth.coo_values(m, *synth.lame(*synth.materials(m.n_elem, s1)))
    A0 = S.coo_assemble(m.n_nodes, m.n_nodes, i, j, v0)
    H = solve.setup(A0, m.coords, m.dirichlet)
    t0 = time.perf_counter()
    A1 = S.coo_assemble(m.n_nodes, m.n_nodes, i, j, v1)
    t_coo = time.perf_counter() - t0
    t0 = time.perf_counter()
    A = A1
    for L in H.levels[:-1]:
        A = S.ptap(A, L.P)
    t_ptap = time.perf_counter() - t0
    H1 = solve.recompute(H, A1)
    b = synth.rhs(m, sb)
    t0 = time.perf_counter()
    _, its, rel, ok = solve.pcg(A1, b, lambda r: solve.vcycle(H1, r), rtol=1e-8)
    t_pcg = time.perf_counter() - t0
    return {"n": n, "dofs": int(m.n_dof), "nnzb": int(A1.nnzb), "levels": [int(L.A.nbr * L.A.br) for L in H.levels],
            "coo_s": t_coo, "ptap_s": t_ptap, "pcg_s": t_pcg, "pcg_its": its, "converged": bool(ok),
            "relres": rel, "host_cpus": os.cpu_count(), "cpu_model": _cpu_model()}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def start_cpu_baseline(n: int):
    """Start the oracle child process (one thread, numerical libraries single-threaded)."""
    env = dict(os.environ)
    for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS", "BLIS_NUM_THREADS"):
        env[k] = "1"
    cmd = [sys.executable, os.path.abspath(__file__), "--cpu-baseline-only", "--cpu-n", str(n)]
    return subprocess.Popen(cmd, env=env, stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)


def finish_cpu_baseline(proc, timeout: float = 600.0) -> dict | None:
    try:
        out, err = proc.communicate(timeout=timeout)
    except subprocess.TimeoutExpired:
        proc.kill()
        proc.communicate()
        log("cpu baseline timed out")
        return None
    if proc.returncode != 0:
        log("cpu baseline failed: " + err[-2000:])
        return None
    return json.loads(out.strip().splitlines()[-1])


# ----------------------------------------------------------------------------------
# GPU benchmark
# ----------------------------------------------------------------------------------
def _time_launches(torch, stream, fn, reps):
    for _ in range(3):
        fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def spmv_probe(B, RL, torch, plan, HA, vals0, n_dof, a_inf, reps, stream):
    """Average durations of the fine 3x3 SpMVs, timed with HIP events on the stream they
    are launched on, with their algorithmic bandwidth: bsr_spmv (every block read) and
    bsr_spmv_sym (the symmetric reads the hierarchy and CG use: diagonal and upper
    blocks from memory, lower blocks as transposed mirrors), in FP64 and on an FP32 copy
    of the operator."""
    B.coo_assemble_blocked(plan, vals0, B.INSERT, HA)
    rp, ci, v = HA.arrays()
    rows = torch.repeat_interleave(torch.arange(a_inf["nbr"], device="cuda"), (rp[1:] - rp[:-1]).long())
    n_lower = int((ci.long() < rows).sum())
    n_upper = a_inf["nnzb"] - n_lower
    del rows
    H32 = B.bsr_create(a_inf["nbr"], a_inf["nbc"], 3, 3, rp, ci, v.to(torch.float32).contiguous())
    del v
    out = {"reps": reps, "n_upper_blocks": n_upper, "n_lower_blocks": n_lower}
    for tag, H, dt, s in (("f64", HA, torch.float64, 8), ("f32", H32, torch.float32, 4)):
        xv = torch.rand(n_dof, dtype=dt, device="cuda")
        yv = torch.zeros(n_dof, dtype=dt, device="cuda")
        ms = _time_launches(torch, stream, lambda: B.bsr_spmv(H, 1.0, xv, 0.0, yv), reps)
        ms_sym = _time_launches(torch, stream, lambda: B.bsr_spmv_sym(H, 1.0, xv, 0.0, yv), reps)
        nb = RL.spmv_bytes(a_inf["nbr"], a_inf["nbc"], 3, 3, a_inf["nnzb"], s, s)
        nb_sym = RL.spmv_sym_bytes(a_inf["nbr"], 3, n_upper, n_lower, s, s)
        out[tag] = {"full": {"avg_launch_ms": ms, "bytes_per_launch": nb, "achieved_GBs": nb / (ms * 1e-3) / 1e9},
                    "sym": {"avg_launch_ms": ms_sym, "bytes_per_launch": nb_sym,
                            "achieved_GBs": nb_sym / (ms_sym * 1e-3) / 1e9,
                            "full_equivalent_GBs": nb / (ms_sym * 1e-3) / 1e9}}
        log(f"[spmv probe] {tag}: full {ms:.3f} ms ({nb / (ms * 1e-3) / 1e9:.0f} GB/s), symmetric reads "
            f"{ms_sym:.3f} ms ({nb_sym / (ms_sym * 1e-3) / 1e9:.0f} GB/s on {nb_sym / 1e9:.2f} GB)")
    del H32
    return out


def copy_probe(torch, stream, nbytes=1 << 30, reps=10):
    """A plain streaming kernel of known size (y = -x, 8-byte elements: nbytes read and
    nbytes written per launch), used to scale hardware byte counters."""
    x = torch.rand(nbytes // 8, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.neg(x, out=y)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        torch.neg(x, out=y)
    e1.record(stream)
    e1.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"bytes_read": nbytes, "bytes_written": nbytes, "avg_launch_ms": ms,
            "GBs": 2 * nbytes / (ms * 1e-3) / 1e9}


def run_batch(args, B, torch, dev, stream):
    """Batch of 24 independent Q1 instances, edge n ~ U{16..48} (rng seed 100), material
    seeds 200+t (redraw 1200+t), 8 right-hand sides each (seed 300+t), FP32
    hierarchies, FP64 CG; one step = assemble + Galerkin recompute + refresh + batched
    CG over all 192 systems with a graph-replayed iteration block."""
    import numpy as np

    import synth

    t0 = time.perf_counter()
    sizes = synth.batch_sizes()
    bt = synth.make_batch(sizes, nrhs=8)
    vals = [synth.batch_values_torch(bt, dev)]
    mats2 = [synth.lame(*synth.materials(m.n_elem, 1200 + t)) for t, m in enumerate(bt["meshes"])]
    vals.append(torch.cat([synth.coo_values_torch(m, lam, mu, dev) for m, (lam, mu) in zip(bt["meshes"], mats2)]))
    b = torch.as_tensor(bt["b"], device=dev)
    n_nodes = bt["n_nodes"]
    n_dof = 3 * n_nodes
    log(f"[batch] {len(sizes)} instances, sizes {sizes.tolist()}, {n_dof} dofs ({time.perf_counter() - t0:.1f}s)")
    plan, HA = B.coo_plan_create(n_nodes, n_nodes, 3, 3, bt["i"], bt["j"])
    B.coo_assemble_blocked(plan, vals[0], B.INSERT, HA)
    del bt["i"], bt["j"]
    res = {"instances": int(len(sizes)), "sizes": sizes.tolist(), "nrhs": 8, "dofs": int(n_dof),
           "fine_nnzb": HA.info()["nnzb"]}
    modes = [("graph", 4)] + ([("eager", 0)] if args.batch_eager else [])
    for name, gi in modes:
        o = B.blkamg_opts_default()
        o.hier_dtype, o.p_dtype = B.F32, B.F32
        o.pcg_graph_iters = gi
        o.autotune_nrhs = 8
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        M = B.amg_setup_batched(HA, bt["row0"], bt["coords"], bt["dirichlet"], o)
        t_setup = time.perf_counter() - t0
        x = torch.zeros_like(b)
        rec = []
        for s in range(args.warmup + args.steps):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
            vi = (s + 1) % 2
            ev[0].record(stream)
            B.coo_assemble_blocked(plan, vals[vi], B.INSERT, HA)
            ev[1].record(stream)
            B.amg_galerkin_recompute(M)
            ev[2].record(stream)
            B.amg_smoother_refresh(M)
            ev[3].record(stream)
            code, its, rel = B.pcg_solve(HA, M, b, x, rtol=1e-8, maxit=1000, nrhs=8)
            ev[4].record(stream)
            ev[4].synchronize()
            ph = [ev[k].elapsed_time(ev[k + 1]) for k in range(4)]
            if s >= args.warmup:
                rec.append({"coo_ms": ph[0], "ptap_ms": ph[1], "refresh_ms": ph[2], "pcg_ms": ph[3],
                            "its_max": int(its.max()), "its_mean": float(its.mean()), "status": code,
                            "relres_max": float(rel.max())})
            log(f"[batch/{name}] step {s}: coo {ph[0]:.2f} ms, ptap {ph[1]:.2f} ms, refresh {ph[2]:.2f} ms, "
                f"pcg {ph[3]:.1f} ms (its {int(its.min())}..{int(its.max())}, relres max {float(rel.max()):.1e})")
        med = {k: statistics.median(r[k] for r in rec) for k in ("coo_ms", "ptap_ms", "refresh_ms", "pcg_ms")}
        res[name] = {"pcg_graph_iters": gi, "setup_s": t_setup, "median_ms": med, "steps": rec,
                     "systems_per_s": 192.0 / (med["pcg_ms"] * 1e-3), "levels": M.num_levels()}
        del M
        torch.cuda.synchronize()
    return res


def run_q2(args, B, RL, torch, dev, stream):
    """Triquadratic (Q2, 27-node) elasticity at q2_n^3 elements: as many dofs as the Q1
    problem with twice the edge (64^3 Q2 and 128^3 Q1 both have 6,440,067 dofs), with
    block rows of 27 to 125 blocks instead of at most 27 (the nonzeros-per-row study of
    paper §4.6, Table 4).  Same material and right-hand-side seeds and the same hot path
    as the Q1 workload; mixed and FP64 hierarchies, then the fine FP64 SpMV probe."""
    import synth

    n = args.q2_n
    t0 = time.perf_counter()
    mesh = synth.make_mesh_q2(n)
    ii, jj = synth.coo_indices(mesh)
    mats = [synth.lame(*synth.materials(mesh.n_elem, 11)), synth.lame(*synth.materials(mesh.n_elem, 1011))]
    vals = [synth.coo_values_torch(mesh, lam, mu, dev) for lam, mu in mats]
    b = torch.as_tensor(synth.rhs(mesh, 12), device=dev)
    log(f"[q2] inputs ready: n={n} dofs={mesh.n_dof} n_coo={len(ii)} ({time.perf_counter() - t0:.1f}s)")
    t0 = time.perf_counter()
    plan, HA = B.coo_plan_create(mesh.n_nodes, mesh.n_nodes, 3, 3, ii, jj)
    t_plan = time.perf_counter() - t0
    del ii, jj
    a_inf = HA.info()
    log(f"[q2] coo plan: nnzb={a_inf['nnzb']} ({t_plan:.1f}s)")
    res = {"n": n, "dofs": mesh.n_dof, "fine_nnzb": a_inf["nnzb"],
           "scalar_nnz_per_row": a_inf["nnzb"] * 9 / mesh.n_dof, "coo_plan_s": t_plan}
    variants = () if args.probe_only else ("mixed", "fp64")  # --probe-only: the SpMV probe alone (counters)
    for var in variants:
        r = run_variant(args, B, RL, torch, dev, stream, var, mesh, plan, HA, a_inf, vals, b, tag=f"q2/{var}")
        r.pop("_x", None)
        res[var] = r
    probe = spmv_probe(B, RL, torch, plan, HA, vals[0], mesh.n_dof, a_inf, args.probe_reps, stream)
    for tag in ("f64", "f32"):
        for mode in ("full", "sym"):
            probe[tag][mode]["frac"] = probe[tag][mode]["achieved_GBs"] / RL.HBM_PEAK_GBS
    res["spmv"] = probe
    p64 = probe["f64"]
    log(f"[q2] fine FP64 SpMV {p64['full']['avg_launch_ms']:.3f} ms ({100 * p64['full']['frac']:.1f}% of HBM peak), "
        f"symmetric reads {p64['sym']['avg_launch_ms']:.3f} ms ({100 * p64['sym']['frac']:.1f}%)")
    del plan, HA, vals
    torch.cuda.synchronize()
    return res


def _event_ms(torch, stream, fn, reps):
    """Average duration of fn() over reps calls, HIP events on the launch stream."""
    for _ in range(2):
        fn()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        fn()
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def run_aggregation(B, torch, HA, dirichlet):
    """Fine-level aggregation of the 128^3 operator's block graph: the device Luby rounds
    (best of 3 calls, each synchronous) against the host greedy pass."""
    import numpy as np

    t_dev = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        agg, n_agg, rounds = B.sa_aggregate_device(HA, dirichlet)
        t_dev.append(time.perf_counter() - t0)
    rp, ci, _ = HA.arrays()
    rp, ci = rp.cpu().numpy(), ci.cpu().numpy()
    t0 = time.perf_counter()
    _, n_host = B.sa_aggregate(rp, ci, np.asarray(dirichlet, dtype=np.uint8))
    t_host = time.perf_counter() - t0
    res = {"device_s": min(t_dev), "rounds": rounds, "device_aggregates": n_agg, "host_greedy_s": t_host,
           "host_aggregates": n_host}
    log(f"[aggregation] device Luby {1e3 * res['device_s']:.1f} ms ({rounds} rounds, {n_agg} aggregates); "
        f"host greedy {1e3 * t_host:.0f} ms ({n_host} aggregates)")
    return res


def run_cold_setup(B, torch, mesh, HA):
    """Cold setup of the FP64 hierarchy at the benchmark size with the Galerkin symbolic
    phase (patterns of A P and A_c, contribution lists, workgroup tables) and the
    smoothed-prolongator pattern built on the device (the default), against the same
    setup with the symbolic phase built on the host (tuning switch host_symbolic); wall
    clock, each synchronous.  Both hierarchies have the same levels and operators."""
    out = {}
    old = os.environ.get("BLKAMG_PTAP_TUNE")
    try:
        for tag, tune in (("device_s", "ap_sort"), ("host_symbolic_s", "ap_sort,host_symbolic")):
            os.environ["BLKAMG_PTAP_TUNE"] = tune
            o = B.blkamg_opts_default()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            M = B.amg_setup(HA, mesh.coords, mesh.dirichlet, o)
            out[tag] = time.perf_counter() - t0
            out.setdefault("levels", M.num_levels())
            del M
            torch.cuda.synchronize()
    finally:
        if old is None:
            os.environ.pop("BLKAMG_PTAP_TUNE", None)
        else:
            os.environ["BLKAMG_PTAP_TUNE"] = old
    out["speedup"] = out["host_symbolic_s"] / out["device_s"]
    log(f"[cold setup] FP64: device symbolic {out['device_s']:.2f} s, host symbolic {out['host_symbolic_s']:.2f} s")
    return out


def run_fe(args, B, torch, dev, stream):
    """Standalone finite-element assembly (the blocked COO primitive's use beyond the
    Galerkin product, paper §5).  Q1 elasticity on a distorted fe_n^3 mesh (interior nodes
    moved by up to 0.2 h, seed 31; materials seed 11): the device element kernel writing
    the blocked COO value stream, blocked COO assembly of that stream, and
    element-by-element assembly without a stream (FP64 atomics; colour passes).  Then, at
    fe_scalar_n^3, the same stream assembled as blocked COO and as scalar COO (1x1 blocks
    at coordinates 3i+c, 3j+d): plan size and assembly time."""
    import numpy as np

    import synth

    reps = max(args.steps, 3)
    res = {}
    for n, scalar in ((args.fe_n, False), (args.fe_scalar_n, True)):
        t0 = time.perf_counter()
        m = synth.make_mesh(n, distort=0.2, seed=31)
        lam, mu = synth.lame(*synth.materials(m.n_elem, 11))
        en = torch.as_tensor(m.elem_nodes.astype(np.int32), device=dev)
        X = torch.as_tensor(m.coords, device=dev)
        lam_t, mu_t = torch.as_tensor(lam, device=dev), torch.as_tensor(mu, device=dev)
        i, j = synth.coo_indices(m)
        vals = torch.empty((m.n_elem * 64 + m.n_dirichlet, 3, 3), dtype=torch.float64, device=dev)
        plan, HA = B.coo_plan_create(m.n_nodes, m.n_nodes, 3, 3, i, j)
        perm, seg = plan.index_map()
        n_valid, nnzb = perm.numel(), seg.numel() - 1
        del perm, seg
        B.fe_q1_stream(en, X, lam_t, mu_t, vals, m.n_dirichlet)  # checks the node range once
        log(f"[fe] n={n}: {m.n_elem} elements, nnzb {nnzb} ({time.perf_counter() - t0:.1f}s)")
        r = {"n": n, "elements": m.n_elem, "stream_blocks": int(vals.shape[0]), "valid_blocks": n_valid,
             "nnzb": nnzb, "coo_plan_bytes": 4 * (n_valid + nnzb + 1)}
        r["element_kernel_ms"] = _event_ms(torch, stream, lambda: B.fe_q1_stream(
            en, X, lam_t, mu_t, vals, m.n_dirichlet, check_nodes=False), reps)
        r["element_kernel_bytes"] = vals.numel() * 8 + m.n_elem * (32 + 16) + m.n_nodes * 24
        r["coo_assemble_ms"] = _event_ms(torch, stream, lambda: B.coo_assemble_blocked(plan, vals, B.INSERT, HA),
                                         reps)
        r["coo_assemble_bytes"] = n_valid * (72 + 4) + (nnzb + 1) * 4 + nnzb * 72
        for k in ("element_kernel", "coo_assemble"):
            r[k + "_GBs"] = r[k + "_bytes"] / (r[k + "_ms"] * 1e-3) / 1e9
        if not scalar:
            ref = HA.arrays()[2].clone()
            P = B.fe_ebe_plan_create(HA, m.elem_nodes, m.dirichlet)
            r.update({("ebe_" + k): v for k, v in P.info().items()})
            for name, mode in (("atomic", B.FE_ATOMIC), ("colored", B.FE_COLORED)):
                r[f"ebe_{name}_ms"] = _event_ms(torch, stream, lambda: B.fe_q1_assemble_ebe(
                    P, HA, en, X, lam_t, mu_t, mode, check_nodes=False), reps)
                got = HA.arrays()[2]
                r[f"ebe_{name}_max_rel_diff"] = float((got - ref).abs().max() / ref.abs().max())
                del got
            r["stream_plus_coo_ms"] = r["element_kernel_ms"] + r["coo_assemble_ms"]
            log(f"[fe] element kernel {r['element_kernel_ms']:.2f} ms ({r['element_kernel_GBs']:.0f} GB/s), "
                f"blocked COO {r['coo_assemble_ms']:.2f} ms ({r['coo_assemble_GBs']:.0f} GB/s); element by "
                f"element: atomic {r['ebe_atomic_ms']:.2f} ms, {r['ebe_n_colors']} colours "
                f"{r['ebe_colored_ms']:.2f} ms")
            del P, ref
            res["assembly"] = r
        else:
            c = np.arange(3, dtype=np.int32)
            isc = np.where(i[:, None, None] >= 0, 3 * i[:, None, None] + c[None, :, None], -1)
            isc = np.broadcast_to(isc, (len(i), 3, 3)).reshape(-1).astype(np.int32)
            jsc = np.where(j[:, None, None] >= 0, 3 * j[:, None, None] + c[None, None, :], -1)
            jsc = np.broadcast_to(jsc, (len(j), 3, 3)).reshape(-1).astype(np.int32)
            t0 = time.perf_counter()
            plan1, H1 = B.coo_plan_create(m.n_dof, m.n_dof, 1, 1, isc, jsc)
            r["scalar_plan_create_s"] = time.perf_counter() - t0
            del isc, jsc
            perm, seg = plan1.index_map()
            nv1, nnz1 = perm.numel(), seg.numel() - 1
            del perm, seg
            r.update({"scalar_valid_entries": nv1, "scalar_nnz": nnz1, "scalar_coo_plan_bytes": 4 * (nv1 + nnz1 + 1)})
            r["scalar_coo_assemble_ms"] = _event_ms(torch, stream, lambda: B.coo_assemble_blocked(
                plan1, vals, B.INSERT, H1), reps)
            r["plan_bytes_ratio"] = r["scalar_coo_plan_bytes"] / r["coo_plan_bytes"]
            r["assemble_time_ratio"] = r["scalar_coo_assemble_ms"] / r["coo_assemble_ms"]
            log(f"[fe] n={n} blocked COO {r['coo_assemble_ms']:.3f} ms, plan {r['coo_plan_bytes'] / 1e6:.0f} MB; "
                f"scalar COO {r['scalar_coo_assemble_ms']:.3f} ms, plan {r['scalar_coo_plan_bytes'] / 1e6:.0f} MB")
            del plan1, H1
            res["blocked_vs_scalar"] = r
        del plan, HA, vals, en, X, lam_t, mu_t
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    return res


def run_learned(args, B, torch, dev, stream):
    """Deployment of the learned eigenbound on Q1 elasticity at learned_n^3 elements
    (material seed 21, redraw 1021, right-hand side seed 22): FP32 hierarchy with
    Lanczos estimates vs FP32 hierarchy with the network, which supplies each level's
    lambda_hat and prolongator-smoothing weight omega from the cold setup on (growth
    test, Lanczos fallback), plus the plain FP64 path.  Each is timed as cold setup
    (wall clock, median of a few setups) and hot steps (assemble + recompute + refresh + PCG to 1e-8);
    lambda errors are taken against 50-step reorthogonalised Lanczos."""
    import numpy as np

    import synth
    from paper_2606_24748_amd import train_eigmlp

    model = train_eigmlp.load_model(args.model or train_eigmlp.DEFAULT_MODEL)
    n = args.learned_n
    mesh = synth.make_mesh(n)
    ii, jj = synth.coo_indices(mesh)
    vals = [synth.coo_values_torch(mesh, *synth.lame(*synth.materials(mesh.n_elem, sd)), dev) for sd in (21, 1021)]
    b = torch.as_tensor(synth.rhs(mesh, 22), device=dev)
    plan, HA = B.coo_plan_create(mesh.n_nodes, mesh.n_nodes, 3, 3, ii, jj)
    del ii, jj
    res = {"n": n, "dofs": mesh.n_dof}
    # one untimed setup first, so that no variant's cold setup pays the process's first
    # kernel loads (the section may run alone)
    B.coo_assemble_blocked(plan, vals[0], B.INSERT, HA)
    o = B.blkamg_opts_default()
    o.hier_dtype, o.p_dtype = B.F32, B.F32
    B.amg_setup(HA, mesh.coords, mesh.dirichlet, o)
    torch.cuda.synchronize()
    for name, hier, eig in (("mixed-lanczos", B.F32, B.EIG_LANCZOS), ("mixed-mlp", B.F32, B.EIG_MLP),
                            ("fp64-lanczos", B.F64, B.EIG_LANCZOS)):
        B.coo_assemble_blocked(plan, vals[0], B.INSERT, HA)
        o = B.blkamg_opts_default()
        o.hier_dtype, o.p_dtype, o.eig_mode = hier, hier, eig
        o.mlp_guard = B.GUARD_PCG  # hot refreshes run no smoother test; CG checks its residual
        keep = B.opts_with_model(o, model) if eig == B.EIG_MLP else None
        # the cold setup's wall clock varies with host work from call to call; the
        # median of a few setups is reported and the last hierarchy is kept
        t_setups, M = [], None
        for _ in range(max(1, args.learned_setups)):
            del M
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            M = B.amg_setup(HA, mesh.coords, mesh.dirichlet, o)
            t_setups.append(time.perf_counter() - t0)
        t_setup = statistics.median(t_setups)
        del keep
        x = torch.zeros_like(b)
        code, its0, rel0 = B.pcg_solve(HA, M, b, x, rtol=1e-8, maxit=1000)  # solve on the setup's own values
        rec = []
        for s in range(args.warmup + args.steps):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
            vi = (s + 1) % 2
            ev[0].record(stream)
            B.coo_assemble_blocked(plan, vals[vi], B.INSERT, HA)
            ev[1].record(stream)
            B.amg_galerkin_recompute(M)
            ev[2].record(stream)
            B.amg_smoother_refresh(M)
            ev[3].record(stream)
            code, its, rel = B.pcg_solve(HA, M, b, x, rtol=1e-8, maxit=1000)
            ev[4].record(stream)
            ev[4].synchronize()
            ph = [ev[k].elapsed_time(ev[k + 1]) for k in range(4)]
            if s >= args.warmup:
                rec.append({"coo_ms": ph[0], "ptap_ms": ph[1], "refresh_ms": ph[2], "pcg_ms": ph[3], "its": its,
                            "status": code, "relres": rel})
            log(f"[learned/{name}] step {s}: refresh {ph[2]:.2f} ms, pcg {ph[3]:.1f} ms ({its} its)")
        med = {k: statistics.median(r[k] for r in rec) for k in ("coo_ms", "ptap_ms", "refresh_ms", "pcg_ms")}
        lam = M.lambdas().tolist()
        judge = B.amg_judge_lambdas(M, 50)[:, 0].tolist()
        s_lam, s_om, s_learned = B.amg_setup_weights(M)
        ent = {"setup_s": t_setup, "setup_s_all": t_setups, "setup_pcg_its": its0, "median_ms": med, "steps": rec, "lambda": lam,
               "lambda_judge": judge, "lambda_rel_err": [a / j - 1.0 for a, j in zip(lam, judge)],
               "setup_lambda": s_lam[:, 0].tolist(), "setup_omega": s_om[:, 0].tolist(),
               "setup_learned": s_learned.tolist(), "iterations": [r["its"] for r in rec],
               "refresh_plus_pcg_ms": med["refresh_ms"] + med["pcg_ms"],
               "hot_step_ms": med["ptap_ms"] + med["refresh_ms"] + med["pcg_ms"],
               "ptap_plus_pcg_ms": med["ptap_ms"] + med["pcg_ms"]}
        ent["setup_plus_hot_step_s"] = t_setup + ent["hot_step_ms"] * 1e-3
        if eig == B.EIG_MLP:
            fb, g, om = B.amg_eig_status(M)
            ent["fallback_levels"] = fb.tolist()
            ent["omega_pred"] = om[:, 0].tolist()
            ent["guard_armed"], ent["guard_restarts"] = B.amg_guard_status(M)
        res[name] = ent
        del M
        torch.cuda.synchronize()
    lz, nn, fp = res["mixed-lanczos"], res["mixed-mlp"], res["fp64-lanczos"]
    res["mlp_vs_lanczos_refresh_speedup"] = lz["median_ms"]["refresh_ms"] / nn["median_ms"]["refresh_ms"]
    res["mlp_vs_lanczos_hot_step_speedup"] = lz["hot_step_ms"] / nn["hot_step_ms"]
    res["mlp_vs_lanczos_setup_plus_hot_step_speedup"] = lz["setup_plus_hot_step_s"] / nn["setup_plus_hot_step_s"]
    res["mlp_minus_lanczos_iterations"] = [a - c for a, c in zip(nn["iterations"], lz["iterations"])]
    res["mixed_mlp_vs_fp64_solve_speedup"] = fp["refresh_plus_pcg_ms"] / nn["refresh_plus_pcg_ms"]
    return res


def variant_opts(B, var):
    """Setup options of a hierarchy variant."""
    o = B.blkamg_opts_default()
    if var == "fp64":
        o.hier_dtype, o.p_dtype = B.F64, B.F64
    elif var == "mixed":
        o.hier_dtype, o.p_dtype = B.F32, B.F32
    elif var == "mixed-mlp":
        o.hier_dtype, o.p_dtype, o.eig_mode = B.F32, B.F32, B.EIG_MLP
        o.mlp_guard = B.GUARD_PCG
    elif var == "mixed-bf16":
        o.hier_dtype, o.p_dtype = B.F32, B.BF16
    elif var == "mixed-luby":
        o.hier_dtype, o.p_dtype, o.agg_mode = B.F32, B.F32, B.AGG_LUBY
    else:
        raise SystemExit(f"unknown variant {var}")
    return o


def run_variant(args, B, RL, torch, dev, stream, var, mesh, plan, HA, a_inf, vals, b, tag=None):
    """Set up one hierarchy variant on the assembled operator and time the hot path
    (assembly, Galerkin recompute, refresh, PCG) over warmup + steps passes."""
    tag = tag or var
    o = variant_opts(B, var)
    keep = None
    if var == "mixed-mlp":  # the network's lambda_hat and omega from the cold setup on
        from paper_2606_24748_amd import train_eigmlp
        keep = B.opts_with_model(o, train_eigmlp.load_model(args.model or train_eigmlp.DEFAULT_MODEL))
    B.coo_assemble_blocked(plan, vals[0], B.INSERT, HA)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    M = B.amg_setup(HA, mesh.coords, mesh.dirichlet, o)
    t_setup = time.perf_counter() - t0
    del keep
    nl = M.num_levels()
    lev = []
    for l in range(nl):
        Al, Pl = M.level(l)
        ai = Al.info()
        lev.append({"nbr": ai["nbr"], "bs": ai["bs_r"], "nnzb": ai["nnzb"],
                    "p_nnzb": Pl.info()["nnzb"] if Pl is not None else 0})
    log(f"[{tag}] setup {t_setup:.1f}s levels {[(d['nbr'] * d['bs'], d['nnzb']) for d in lev]}")
    x = torch.zeros(mesh.n_dof, dtype=torch.float64, device=dev)
    rec = []
    for s in range(args.warmup + args.steps):
        timed = s >= args.warmup
        if s == args.warmup:
            torch.cuda.synchronize()
            t_region = time.perf_counter()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
        vi = (s + 1) % 2
        ev[0].record(stream)
        B.coo_assemble_blocked(plan, vals[vi], B.INSERT, HA)
        ev[1].record(stream)
        B.amg_galerkin_recompute(M)
        ev[2].record(stream)
        B.amg_smoother_refresh(M)
        ev[3].record(stream)
        code, its, rel = B.pcg_solve(HA, M, b, x, rtol=1e-8, maxit=1000)
        ev[4].record(stream)
        ev[4].synchronize()
        ph = [ev[k].elapsed_time(ev[k + 1]) for k in range(4)]
        if timed:
            rec.append({"coo_ms": ph[0], "ptap_ms": ph[1], "refresh_ms": ph[2], "pcg_ms": ph[3], "its": its,
                        "relres": rel, "status": code, "values": vi})
        log(f"[{tag}] step {s} {'timed' if timed else 'warmup'}: coo {ph[0]:.2f} ms, ptap {ph[1]:.2f} ms, "
            f"refresh {ph[2]:.2f} ms, pcg {ph[3]:.1f} ms ({its} its, relres {rel:.2e})")
    torch.cuda.synchronize()
    region_s = time.perf_counter() - t_region
    # true residual of the last solve with the FP64 fine operator (library SpMV)
    r = b.clone()
    B.bsr_spmv(HA, -1.0, x, 1.0, r)
    true_rel = float(torch.linalg.norm(r) / torch.linalg.norm(b))
    med = {k: statistics.median(rr[k] for rr in rec) for k in ("coo_ms", "ptap_ms", "refresh_ms", "pcg_ms")}
    # Galerkin recompute algorithmic bytes over all levels
    vsz = 8 if o.hier_dtype == B.F64 else 4
    psz = {B.F64: 8, B.F32: 4, B.BF16: 2}[o.p_dtype]
    ptap_bytes = 0
    ptap_flops = 0  # the products the recompute executes (its plans' pair counts)
    for l in range(nl - 1):
        d, c = lev[l], lev[l + 1]
        ptap_bytes += RL.ptap_bytes(d["nbr"], d["nnzb"], d["bs"], d["p_nnzb"], 6, c["nbr"], c["nnzb"], vsz, psz)
        pi = B.ptap_plan_info(M.level(l + 1)[0])
        if ptap_flops is not None and pi["ap_pairs"] >= 0 and pi["c_pairs"] >= 0:
            ptap_flops += RL.ptap_flops(pi["ap_pairs"], pi["c_pairs"], d["bs"], 6)
        else:
            ptap_flops = None
    res = {
        "setup_s": t_setup, "levels": lev, "steps": rec, "median_ms": med,
        "pcg_plus_ptap_s": (med["pcg_ms"] + med["ptap_ms"]) / 1e3,
        "ms_per_step": region_s * 1e3 / max(args.steps, 1),
        "iterations": [rr["its"] for rr in rec], "true_relres": true_rel,
        "ptap_alg_GBs": ptap_bytes / (med["ptap_ms"] * 1e-3) / 1e9,
        "ptap_alg_bytes": ptap_bytes,
        "ptap_flops": ptap_flops,
        "pcg_iter_bytes": RL.pcg_iteration_bytes(lev, vsz, psz),
        "x_norm": float(torch.linalg.norm(x)),
    }
    res["_x"] = x
    res["lambdas"] = M.lambdas().tolist()
    if var == "mixed-mlp":
        fb, g, _ = B.amg_eig_status(M)
        res["fallback_levels"] = fb.tolist()
        res["growth"] = g[:, 0].tolist()
    del M
    torch.cuda.synchronize()
    return res


def run_config_s(args, B, RL, torch, dev, stream):
    """The 64^3 FP64 problem the CPU baseline runs (823,875 dofs, materials seed 1,
    redraw 1001, right-hand side seed 2): the same hot path on the GPU, so the oracle's
    time has a like-for-like GPU figure beside it."""
    import synth

    n = args.cpu_n
    s0, s1, sb = CPU_SEEDS
    mesh = synth.make_mesh(n)
    ii, jj = synth.coo_indices(mesh)
    vals = [synth.coo_values_torch(mesh, *synth.lame(*synth.materials(mesh.n_elem, sd)), dev) for sd in (s0, s1)]
    b = torch.as_tensor(synth.rhs(mesh, sb), device=dev)
    plan, HA = B.coo_plan_create(mesh.n_nodes, mesh.n_nodes, 3, 3, ii, jj)
    del ii, jj
    r = run_variant(args, B, RL, torch, dev, stream, "fp64", mesh, plan, HA, HA.info(), vals, b, tag=f"S{n}/fp64")
    r.pop("_x", None)
    r["n"], r["dofs"] = n, mesh.n_dof
    del plan, HA, vals
    torch.cuda.synchronize()
    return r


def run_ptap_only(args, B, RL, torch, dev, stream):
    """Galerkin recompute alone (for counter runs): the fine operator at n^3, the first
    hierarchy variant, then `steps` recomputes on alternating material draws."""
    import synth

    n = args.n
    mesh = synth.make_mesh(n)
    ii, jj = synth.coo_indices(mesh)
    vals = [synth.coo_values_torch(mesh, *synth.lame(*synth.materials(mesh.n_elem, sd)), dev) for sd in (11, 1011)]
    plan, HA = B.coo_plan_create(mesh.n_nodes, mesh.n_nodes, 3, 3, ii, jj)
    del ii, jj
    var = [v.strip() for v in args.variants.split(",") if v.strip()][0]
    o = variant_opts(B, var)
    B.coo_assemble_blocked(plan, vals[0], B.INSERT, HA)
    M = B.amg_setup(HA, mesh.coords, mesh.dirichlet, o)
    ms = []
    for s in range(args.warmup + args.steps):
        B.coo_assemble_blocked(plan, vals[(s + 1) % 2], B.INSERT, HA)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        B.amg_galerkin_recompute(M)
        e1.record(stream)
        e1.synchronize()
        if s >= args.warmup:
            ms.append(e0.elapsed_time(e1))
        log(f"[ptap/{var}] step {s}: {e0.elapsed_time(e1):.3f} ms")
    return {"variant": var, "n": n, "ptap_ms": ms, "median_ms": statistics.median(ms) if ms else None}


def _pcg_roofline(RL, r):
    """PCG over the median timed solve: iterations x the iteration byte model."""
    its = [rr["its"] for rr in r["steps"]]
    ms = [rr["pcg_ms"] for rr in r["steps"]]
    per = [r["pcg_iter_bytes"] * i / (t * 1e-3) / 1e9 for i, t in zip(its, ms)]
    ach = statistics.median(per)
    return {"bound": "hbm", "achieved": ach, "peak": RL.HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / RL.HBM_PEAK_GBS,
            "bytes_per_iteration": r["pcg_iter_bytes"], "iterations": statistics.median(its)}


def _ptap_roofline(RL, r, fp64=False):
    """Galerkin recompute over all levels against the HBM roofline: the algorithmic bytes
    of the recompute (A and P read once, A_c written once, int32 indices; no cast of the
    fine operator) over the median recompute time; traffic from the recorded counters
    (FP64 hierarchy only).  Beside it the vector-ALU bound: the block products the
    plans execute (2 bs bs 6 flops per A P pair, 2 6 bs 6 per R (A P) pair) against the
    FP64 (or FP32) vector peak."""
    ms = r["median_ms"]["ptap_ms"]
    ach = r["ptap_alg_bytes"] / (ms * 1e-3) / 1e9
    out = {"bound": "hbm", "achieved": ach, "peak": RL.HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / RL.HBM_PEAK_GBS,
           "traffic": measured_traffic(PTAP_TRAFFIC_RECORD, PTAP_TRAFFIC_SOURCES) if fp64 else None,
           "kernel": "ptap_numeric, all levels", "bytes_per_recompute": r["ptap_alg_bytes"],
           "median_ms": ms}
    if out["traffic"]:
        out["traffic_GBs"] = out["traffic"] / (ms * 1e-3) / 1e9
        out["traffic_frac"] = out["traffic_GBs"] / RL.HBM_PEAK_GBS
    if r.get("ptap_flops"):
        tf = r["ptap_flops"] / (ms * 1e-3) / 1e12
        pk = RL.FP64_PEAK_TFLOPS if fp64 else RL.FP32_PEAK_TFLOPS
        out["valu"] = {"flops": r["ptap_flops"], "achieved": tf, "peak": pk, "unit": "TFLOP/s", "frac": tf / pk}
    return out


def main(argv=None):
    args = parse_args(argv)
    if args.cpu_baseline_only:
        print(json.dumps(cpu_baseline_child(args.cpu_n)))
        return 0
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); this solve-phase build has no "
              "multi-GPU path", file=sys.stderr)
        return 2
    import numpy as np  # noqa: F401
    import torch

    import synth
    from paper_2606_24748_amd import blkamg as B
    from paper_2606_24748_amd import roofline as RL

    assert torch.cuda.is_available(), "no GPU visible"
    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    if args.only_section:
        stream = torch.cuda.current_stream()
        if args.only_section == "q2":
            result = run_q2(args, B, RL, torch, dev, stream)
        elif args.only_section == "fe":
            result = run_fe(args, B, torch, dev, stream)
        elif args.only_section == "ptap":
            result = run_ptap_only(args, B, RL, torch, dev, stream)
        else:
            run = run_learned if args.only_section == "learned" else run_batch
            result = run(args, B, torch, dev, stream)
        print(json.dumps({"section": args.only_section, "result": result}))
        return 0
    cpu_proc = None
    if not args.no_cpu_baseline and not args.probe_only:
        log(f"cpu baseline started (oracle, 1 core, {args.cpu_n}^3)")
        cpu_proc = start_cpu_baseline(args.cpu_n)
    n = args.n
    t_all = time.perf_counter()
    mesh = synth.make_mesh(n)
    ii, jj = synth.coo_indices(mesh)
    mats = [synth.lame(*synth.materials(mesh.n_elem, 11)), synth.lame(*synth.materials(mesh.n_elem, 1011))]
    vals = [synth.coo_values_torch(mesh, lam, mu, dev) for lam, mu in mats]
    b = torch.as_tensor(synth.rhs(mesh, 12), device=dev)
    log(f"inputs ready: n={n} dofs={mesh.n_dof} n_coo={len(ii)} ({time.perf_counter() - t_all:.1f}s)")

    t0 = time.perf_counter()
    plan, HA = B.coo_plan_create(mesh.n_nodes, mesh.n_nodes, 3, 3, ii, jj)
    t_plan = time.perf_counter() - t0
    a_inf = HA.info()
    log(f"coo plan: nnzb={a_inf['nnzb']} ({t_plan:.1f}s)")
    # the same plan built on the device from device coordinates (best of 3, each sync)
    di, dj = torch.as_tensor(ii, device=dev), torch.as_tensor(jj, device=dev)
    t_dplan = []
    for _ in range(3):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dplan, dHA = B.coo_plan_create(mesh.n_nodes, mesh.n_nodes, 3, 3, di, dj)
        t_dplan.append(time.perf_counter() - t0)
        same = dHA.info()["nnzb"] == a_inf["nnzb"]
        del dplan, dHA
    plan_dev = {"device_s": min(t_dplan), "host_s": t_plan, "same_nnzb": bool(same), "entries": int(len(ii))}
    log(f"coo plan on the device: {1e3 * min(t_dplan):.1f} ms (host {1e3 * t_plan:.0f} ms)")
    del ii, jj, di, dj
    torch.cuda.empty_cache()

    stream = torch.cuda.current_stream()
    if args.probe_only:
        probe = spmv_probe(B, RL, torch, plan, HA, vals[0], mesh.n_dof, a_inf, args.probe_reps, stream)
        probe["copy"] = copy_probe(torch, stream)
        print(json.dumps({"probe": probe, "n": n}))
        return 0
    variants = [v.strip() for v in args.variants.split(",") if v.strip()]
    results = {}
    for var in variants:
        results[var] = run_variant(args, B, RL, torch, dev, stream, var, mesh, plan, HA, a_inf, vals, b)

    probe = spmv_probe(B, RL, torch, plan, HA, vals[0], mesh.n_dof, a_inf, args.probe_reps, stream)
    copy = copy_probe(torch, stream)
    aggregation = run_aggregation(B, torch, HA, mesh.dirichlet)
    cold_setup = run_cold_setup(B, torch, mesh, HA)
    side = {}
    del plan, HA, vals
    torch.cuda.empty_cache()
    if not args.no_config_s:
        side["config_s"] = run_config_s(args, B, RL, torch, dev, stream)
        torch.cuda.empty_cache()
    if not args.no_fe:
        side["fe"] = run_fe(args, B, torch, dev, stream)
        torch.cuda.empty_cache()
    if not args.no_q2:
        side["q2"] = run_q2(args, B, RL, torch, dev, stream)
        torch.cuda.empty_cache()
    if not args.no_learned:
        side["learned"] = run_learned(args, B, torch, dev, stream)
        torch.cuda.empty_cache()
    if not args.no_batch:
        side["batch"] = run_batch(args, B, torch, dev, stream)
    # the roofline kernel: the fine FP64 SpMV with symmetric reads, the one CG and the
    # FP64 V-cycle run.  Its achieved rate is the SpMV's algorithmic bytes (every block
    # once, the model the method is measured on) over its duration; it reads only the
    # upper triangle from HBM (own_min_bytes), the lower blocks through the caches, which
    # the counter traffic shows.  The full-read kernel is reported beside it.
    psym, pfull = probe["f64"]["sym"], probe["f64"]["full"]
    spmv_b, spmv_ms = pfull["bytes_per_launch"], psym["avg_launch_ms"]
    achieved = spmv_b / (spmv_ms * 1e-3) / 1e9

    head = "fp64" if "fp64" in results else variants[0]
    hr = results[head]
    cpu = None
    if cpu_proc is not None:
        log("waiting for the cpu baseline")
        cb = finish_cpu_baseline(cpu_proc)
        if cb:
            cs = side.get("config_s")
            gpu_s = cs["pcg_plus_ptap_s"] if cs else None
            cpu = {"value": cb["ptap_s"] + cb["pcg_s"], "unit": "s", "cores": 1, "kind": "oracle",
                   "sample": (f"oracle (numpy/scipy, FP64) on one core of this host ({cb['cpu_model']}): Q1 "
                              f"elasticity {cb['n']}^3 elements ({cb['dofs']} dofs, levels {cb['levels']}), PtAP "
                              f"recompute over all levels {cb['ptap_s']:.1f} s + PCG to 1e-8 {cb['pcg_s']:.1f} s "
                              f"({cb['pcg_its']} its); measured once, not scaled to {n}^3"),
                   "workload_n": cb["n"], "gpu_fp64_same_workload_s": gpu_s,
                   "gpu_speedup_same_workload": (cb["ptap_s"] + cb["pcg_s"]) / gpu_s if gpu_s else None,
                   "pcg_its_oracle": cb["pcg_its"],
                   "pcg_its_gpu": (statistics.median(cs["iterations"]) if cs else None)}
            side["cpu_baseline_measured"] = cb
    for v in results.values():
        v.pop("_x", None)
    value = hr["pcg_plus_ptap_s"]
    out = {
        "metric": METRIC, "value": value, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": hr["ms_per_step"], "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if head == "fp64" else "f32+f64", "data": "synthetic",
        "config": {"workload": f"Q1 elasticity {n}^3 elements ({mesh.n_dof} dofs), lognormal E, "
                               f"{len(hr['levels'])}-level SA, Chebyshev(2) V-cycle PCG to 1e-8",
                   "n": n, "dofs": mesh.n_dof, "variant": head},
        "pcg_ms": hr["median_ms"]["pcg_ms"], "ptap_ms": hr["median_ms"]["ptap_ms"],
        "pcg_its": statistics.median(hr["iterations"]),
        "pcg_ms_range": [min(rr["pcg_ms"] for rr in hr["steps"]), max(rr["pcg_ms"] for rr in hr["steps"])],
        "ptap_ms_range": [min(rr["ptap_ms"] for rr in hr["steps"]), max(rr["ptap_ms"] for rr in hr["steps"])],
        # the whole solve against the HBM roofline, on the iteration byte model of the
        # method (every operator block read once per SpMV, as the paper accounts)
        "pcg_roofline": _pcg_roofline(RL, hr),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": RL.HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / RL.HBM_PEAK_GBS, "traffic": measured_traffic(),
                     "kernel": ("bsr_spmv_sym fine 3x3 f64, symmetric reads "
                                "(spmv_kernel<3,3,1,16,2,double,double,double,EpiAxpby,true>)"),
                     "bytes_per_launch": spmv_b, "avg_launch_ms": spmv_ms,
                     "own_min_bytes": psym["bytes_per_launch"],
                     "own_min_frac": psym["achieved_GBs"] / RL.HBM_PEAK_GBS,
                     "full_reads": {"avg_launch_ms": pfull["avg_launch_ms"], "bytes_per_launch": pfull["bytes_per_launch"],
                                    "frac": pfull["achieved_GBs"] / RL.HBM_PEAK_GBS}},
        "ptap_roofline": _ptap_roofline(RL, hr, fp64=head == "fp64"),
        "copy_GBs": copy["GBs"],
        "coo_plan_ms": {"host": 1e3 * t_plan, "device": 1e3 * plan_dev["device_s"]},
        "cold_setup_s": {"device": cold_setup["device_s"], "host_symbolic": cold_setup["host_symbolic_s"]},
        "cpu_baseline": cpu,
    }
    rl = out["roofline"]
    if rl["traffic"]:  # the counters' bytes over the same duration: what the kernel really moved
        rl["traffic_GBs"] = rl["traffic"] / (spmv_ms * 1e-3) / 1e9
        rl["traffic_frac"] = rl["traffic_GBs"] / RL.HBM_PEAK_GBS
    alt = {}
    for var, r in results.items():
        if var == head:
            continue
        alt[var] = {"value": r["pcg_plus_ptap_s"], "pcg_ms": r["median_ms"]["pcg_ms"],
                    "ptap_ms": r["median_ms"]["ptap_ms"], "pcg_its": statistics.median(r["iterations"]),
                    "speedup_vs_head": value / r["pcg_plus_ptap_s"]}
        if var == "mixed":
            alt[var]["ptap_roofline_frac"] = _ptap_roofline(RL, r)["frac"]
    out["variants"] = alt
    if "mixed" in results and head == "fp64":
        out["mixed_value"] = results["mixed"]["pcg_plus_ptap_s"]
        out["mixed_speedup_vs_fp64"] = value / results["mixed"]["pcg_plus_ptap_s"]
    detail = {"variants": results, "spmv_probe": probe, "copy": copy, "aggregation": aggregation,
              "cold_setup": cold_setup,
              "coo_plan_s": t_plan, "coo_plan": plan_dev, **side}
    line = json.dumps(detail)
    print("[bench] detail " + line, file=sys.stderr, flush=True)
    if args.detail_out:
        with open(args.detail_out, "w") as f:
            f.write(line + "\n")
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
