"""Benchmark of the batched leaf-box reduction (two-level HPS, a1..a4) on one MI355X.

Workload: 16 x 16 x 16 leaf boxes on [0,1]^3, p = 16 (2744 interior nodes per
box), kappa = 40, b = 1 + 0.3 * (8 seeded Gaussian bumps), plane-wave Dirichlet
data, f = 0 (seeded synthetic inputs, workloads.config3).  One step = the whole
hot path over all 4096 boxes: operator assembly, LU, solves with FP64
refinement, DtN/load assembly into the BSR interface matrix, and the diagonal
block reduction.  Inputs (b, g) are resident in HBM before timing starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--nbox N] [--no-fp64] [--no-cpu]

Prints one JSON line.  value = leaf boxes/s of the FP32+IR path.
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

METRIC = "leaf boxes/s + % MFMA peak at p=16; FP32+IR vs FP64 path at <=1e-9 rel err"
PEAK_FP32_MFMA = 157.3e12
PEAK_FP64_MFMA = 78.6e12
PEAK_HBM = 8.0e12


def log(*a):
    print(*a, file=sys.stderr, flush=True)


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_16x16x16_p16.md")
KERNEL_SOURCES = ("paper_2503_04033_amd/csrc/common.h", "paper_2503_04033_amd/csrc/lu.hip")


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the rocprofv3 FETCH_SIZE/WRITE_SIZE summary
    (lines `traffic_bytes_per_launch[<kernel>]: <bytes>`), or None when the summary is
    missing, does not list the kernel, or the kernel sources changed since the counters
    were taken (`kernel_sources_sha256`)."""
    import hashlib
    try:
        kv = {}
        for line in open(TRAFFIC_FILE):
            if ":" in line and not line.startswith(("#", "|", " ")):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        h = hashlib.sha256()
        for src in KERNEL_SOURCES:
            with open(os.path.join(ROOT, src), "rb") as fh:
                h.update(fh.read())
        if kv.get("kernel_sources_sha256") != h.hexdigest():
            return None
        return float(kv[f"traffic_bytes_per_launch[{kernel}]"])
    except (OSError, KeyError, ValueError):
        return None


def host_cpu() -> dict:
    """Model name and logical CPU count of the host (for the CPU baseline record)."""
    model = None
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"model": model, "logical_cpus": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None}


def solve_stage(torch, prob, precision: str, interface: str) -> dict:
    """Build and solve stages end to end on a grid whose interface system also fits the host
    (paper Alg. 1 and Alg. 2): GPU build (a1-a4), factorization of the interface matrix
    (interface 'gpu': nested dissection with dense fronts in HBM; 'host': copy of T and LAPACK
    on the host cores), interface solve, and the GPU interiors with the solve stage's outer
    refinement (FP32+IR).  Wall-clock seconds per part; inputs resident in HBM."""
    from paper_2503_04033_amd import interface as itf
    from paper_2503_04033_amd.nested import NestedDissection
    from paper_2503_04033_amd.solver import TwoLevelSolver
    s = TwoLevelSolver.for_problem(prob, precision=precision, interface=interface)
    bv, fv, gv, _, _ = s.sample(prob.b, prob.f, prob.g)
    br = s.build(bv, fv, gv)  # warm-up (kernel loading, allocator)
    if interface == "gpu":
        s.interface_solver(br)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    br = s.build(bv, fv, gv)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    if interface == "gpu":
        isolver = NestedDissection(s.layout, s.device)
        t2 = time.perf_counter()
        isolver.factor(br.T_vals)
        torch.cuda.synchronize()
        method, mem = "gpu nested dissection", isolver.memory_bytes()
    else:
        T_host = br.T_vals.cpu().numpy()
        t2 = time.perf_counter()
        isolver = itf.InterfaceSolver(s.layout, T_host)
        method, mem = "host " + isolver.method, None
    t3 = time.perf_counter()
    u_face, ub, ui, _ = s.solve(br, gv, isolver, b=bv, f=fv)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    return {"precision": precision, "interface": method, "nbox": s.nbox,
            "interface_unknowns": int(s.layout.nunknown), "interface_device_bytes": mem, "keep": s.keep,
            "chunk": s.chunk, "refine_rounds": s.refine, "build_s": round(t1 - t0, 4),
            "interface_setup_s": round(t2 - t1, 4), "interface_factor_s": round(t3 - t2, 4),
            "solve_stage_s": round(t4 - t3, 4), "end_to_end_s": round(t4 - t0, 4), "u_i": ui, "u_face": u_face,
            "interior_fp64_boxes": len(br.extra.get("interior_fp64", [])),
            "build_fp64_fallback_boxes": len(br.extra.get("fp64_fallback", []))}


def time_stepping(torch, pp, precision: str, nsteps: int) -> dict:
    """Crank-Nicolson stepping (paper Sec. 4.4): setup (leaf factorizations and the GPU
    interface factorization, once) and the per-step time (right-hand side, loads, interface
    solve, interiors), device-synchronized wall clock."""
    from paper_2503_04033_amd.stepping import CrankNicolson
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cn = CrankNicolson(pp, precision)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    cn.step()  # first step (allocator warm-up)
    torch.cuda.synchronize()
    times = []
    for _ in range(nsteps):
        a = time.perf_counter()
        cn.step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - a)
    return {"precision": precision, "nbox": pp.nbox, "p": pp.p, "interface_unknowns": int(cn.s.layout.nunknown),
            "setup_s": round(t1 - t0, 4), "step_ms_median": round(1e3 * float(np.median(times)), 3),
            "step_ms_min": round(1e3 * min(times), 3), "steps": nsteps,
            "refine_rounds": cn.s.refine}


def adjoint_timing(torch, reps: int = 3) -> dict:
    """Forward solve and misfit gradient dJ/db (FP64) at the configuration-5 size, 8x8x8
    boxes, p = 10, kappa = 15, 500 observation nodes: device-synchronized wall clock of the
    forward pass (build, GPU interface factorization, solve, interiors) and of the backward
    pass (transposed box solves, transposed interface solve, gradient), median of reps."""
    import workloads as W
    from paper_2503_04033_amd.adjoint import AdjointSolve
    from paper_2503_04033_amd.solver import TwoLevelSolver
    inv = W.config5()
    prob = inv.forward
    s = TwoLevelSolver.for_problem(prob, precision="fp64", interface="gpu")
    bv, fv, gv, xi, _ = s.sample(prob.b, prob.f, prob.g)
    m = prob.p - 2
    t, i, j, k = inv.obs_nodes.T
    tl = torch.tensor(np.stack([t, (i - 1) + m * (j - 1) + m * m * (k - 1)], axis=1), device=s.device)
    fw, bw = [], []
    for _ in range(reps + 1):
        torch.cuda.synchronize()
        a = time.perf_counter()
        adj = AdjointSolve(s)
        u, _ = adj.forward(bv, fv, gv)
        torch.cuda.synchronize()
        b0 = time.perf_counter()
        w = torch.zeros_like(u)
        w[tl[:, 0], tl[:, 1]] = u[tl[:, 0], tl[:, 1]]  # dJ/du of 0.5 |P u|^2
        adj.gradient(w)
        torch.cuda.synchronize()
        c = time.perf_counter()
        fw.append(b0 - a)
        bw.append(c - b0)
    return {"workload": "8x8x8 boxes, p=10, kappa=15, 500 observation nodes (FP64)", "nbox": prob.nbox,
            "interface_unknowns": int(s.layout.nunknown), "resident_factors": adj.resident,
            "forward_s_median": round(float(np.median(fw[1:])), 4),
            "gradient_s_median": round(float(np.median(bw[1:])), 4)}


def batch_config4(torch, reps: int = 3) -> dict:
    """Three independent problems in one captured stream (12^3 boxes p=8 kappa=10, 8^3 p=12
    kappa=20, 6^3 p=16 kappa=30; FP32+IR): device time of a graph replay with the size groups
    back to back, and with each group on its own stream (parallel graph branches)."""
    import workloads as W
    from paper_2503_04033_amd.batch import BatchedLeafReduction
    probs = W.config4()
    nbox = sum(p.nbox for p in probs)
    out = {"workload": "; ".join(f"{p.nboxes[0]}^3 boxes p={p.p} kappa={p.kappa:g}" for p in probs),
           "nbox": nbox}
    ref = None
    for mode in ("sequential", "concurrent"):
        br = BatchedLeafReduction(probs, "fp32_ir", hbm_budget=64e9)
        for q, pr in enumerate(probs):
            br.sample_inputs(q, pr)
        br.allocate()
        br.capture(concurrent=(mode == "concurrent"))
        br.run()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            br.run()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        vals = [g.T_vals.clone() for g in br.groups]
        if ref is None:
            ref = vals
        else:
            out["concurrent_bitwise_equal"] = all(torch.equal(a, b) for a, b in zip(ref, vals))
        out[mode] = {"ms": round(ms, 3), "boxes_per_s": round(nbox / (ms / 1e3), 1),
                     "chunks": [g.chunk for g in br.groups]}
        del br
        torch.cuda.empty_cache()
    return out


class Runner:
    """Buffers and the per-chunk ABI call sequence for one precision."""

    def __init__(self, prob, precision, nbox, chunk, ir_max_iter=3, ir_tol=1e-12, streams=1):
        import torch
        from paper_2503_04033_amd import interface as itf
        from paper_2503_04033_amd.leaf import LeafPlan
        self.torch = torch
        self.prob = prob
        self.nbox = nbox
        self.plan = LeafPlan(prob.p, prob.h, prob.kappa, precision, ir_max_iter, ir_tol)
        self.info = self.plan.info
        self.layout = itf.build_layout(prob.nboxes, self.info.m)
        self.chunk = min(chunk, nbox)
        dev = torch.device("cuda")
        i = self.info
        mm = i.m * i.m
        self.T_vals = torch.zeros(self.layout.nslot_total * mm * mm + 1, dtype=torch.float64, device=dev)
        self.g_loads = torch.zeros(nbox, i.n_b, dtype=torch.float64, device=dev)
        self.infov = torch.zeros(nbox, dtype=torch.int32, device=dev)
        self.iters = torch.zeros(nbox, dtype=torch.int32, device=dev)
        self.berr = torch.zeros(nbox, dtype=torch.float64, device=dev)
        # one buffer set per stream; chunk j runs on stream j % streams so that the pivoted
        # panels of one chunk overlap the GEMMs of the next
        self.streams = [torch.cuda.Stream() for _ in range(streams)] if streams > 1 else None
        self.bufsets = [self.plan.alloc(self.chunk, dev) for _ in range(max(streams, 1))]
        self.slot_map = torch.tensor(self.layout.slot_map[:nbox], device=dev).contiguous()
        self.triples = torch.tensor(self.layout.reduce_triples, device=dev)
        self.ev = {k: [] for k in ("operators", "factor", "dtn")}

    def step(self, b, g_dir, record=False):
        torch = self.torch
        plan, C = self.plan, self.chunk
        main = torch.cuda.current_stream()
        if self.streams:
            for s in self.streams:
                s.wait_stream(main)
        for j, c0 in enumerate(range(0, self.nbox, C)):
            if self.streams:
                with torch.cuda.stream(self.streams[j % len(self.streams)]):
                    self._chunk(j, c0, b, g_dir, record)
            else:
                self._chunk(j, c0, b, g_dir, record)
        if self.streams:
            for s in self.streams:
                main.wait_stream(s)
        self._reduce()

    def _chunk(self, j, c0, b, g_dir, record):
        torch = self.torch
        plan, C = self.plan, self.chunk
        B = self.bufsets[j % len(self.bufsets)]
        nb = min(C, self.nbox - c0)
        sl = slice(c0, c0 + nb)
        e = [torch.cuda.Event(enable_timing=True) for _ in range(4)] if record else None
        if record:
            e[0].record()
        plan.hps_leaf_operators(nb, b[sl], B["A"], B["anorm"])
        if record:
            e[1].record()
        plan.hps_leaf_factor(nb, B["A"], B["perm"], B["dinv"], self.infov[sl])
        if record:
            e[2].record()
        plan.hps_leaf_dtn(nb, B["A"], B["perm"], B["dinv"], b[sl], B["anorm"], None, g_dir[sl],
                          self.slot_map[sl], self.T_vals, self.g_loads[sl], B["X"], self.iters[sl],
                          self.berr[sl], B["ws"])
        if record:
            e[3].record()
            self.ev["operators"].append((e[0], e[1], nb))
            self.ev["factor"].append((e[1], e[2], nb))
            self.ev["dtn"].append((e[2], e[3], nb))

    def _reduce(self):
        if self.triples.shape[0] and self.nbox == self.prob.nbox:
            from paper_2503_04033_amd.leaf import hps_interface_reduce
            mm = self.info.m ** 2
            hps_interface_reduce(self.triples, mm * mm, self.T_vals)

    def phase_ms(self):
        out = {}
        for k, lst in self.ev.items():
            tot = sum(a.elapsed_time(b) for a, b, _ in lst)
            out[k] = {"ms_total": tot, "launches": len(lst), "boxes": sum(n for _, _, n in lst)}
        return out


def cpu_baseline(prob, nsample: int, seed: int = 0) -> dict:
    """The oracle (plain FP64 NumPy/SciPy) on a bounded sample of boxes of the same workload."""
    from threadpoolctl import threadpool_info

    from oracle import leaf as ol
    rng = np.random.default_rng(seed)
    ids = rng.choice(prob.nbox, size=nsample, replace=False)
    org = prob.box_origins()
    t0 = time.perf_counter()
    for t in ids:
        xi, _ = ol.box_node_coords(org[t], prob.h, prob.p)
        blk = ol.local_blocks(prob.p, prob.h, prob.kappa, prob.b(xi))
        ol.leaf_reduce(blk, prob.f(xi))
    dt = time.perf_counter() - t0
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    return {"value": nsample / dt, "unit": "boxes/s", "cores": int(threads), "kind": "oracle", "host": host_cpu(),
            "sample": f"{nsample} seeded boxes of the same 16^3 p=16 workload (operator + dense LU + "
                      f"{prob.p - 2}^3-row solve with {6 * (prob.p - 2) ** 2 + 1} right-hand sides + DtN), "
                      f"{dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--nbox", type=int, default=0, help="time only the first N boxes (profiling)")
    ap.add_argument("--chunk", type=int, default=2048,
                    help="boxes per launch of the FP32+IR headline (the FP64 leg takes at most 1024: its "
                         "buffers are twice as large)")
    ap.add_argument("--streams", type=int, default=1,
                    help="chunks interleaved over this many HIP streams (each with its own buffers); more "
                         "than one overlaps kernels, so per-kernel event times then include the overlap")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-solve-stage", action="store_true",
                    help="skip the end-to-end build + solve timing at 4x4x4 boxes, p = 16")
    ap.add_argument("--cpu-sample", type=int, default=24)
    ap.add_argument("--ir-max-iter", type=int, default=3)
    ap.add_argument("--ir-tol", type=float, default=1e-12)
    ap.add_argument("--tune", action="append", default=[], metavar="KEY=VALUE",
                    help="plan knob of the FP32+IR headline plan (trsm_schedule, trsm_waves, residual_cols)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run three device-to-device copies of MIB MiB (HBM counter calibration)")
    a = ap.parse_args()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the leaf reduction shards by boxes with no exchange, and this "
              "build runs on a single MI355X (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import torch

    if a.copy_calibration:
        # a plain copy of known size: FETCH_SIZE and WRITE_SIZE of its kernel should each read
        # MIB * 1024 KiB; the ratio scales the counters of the leaf-reduction kernels
        n = a.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_mib": a.copy_calibration, "kib_per_copy": a.copy_calibration * 1024}))
        return

    import workloads as W
    prob = W.config3()
    nbox = a.nbox if a.nbox else prob.nbox
    dev = torch.device("cuda")
    log(f"workload {prob.name}: nbox={nbox} p={prob.p} kappa={prob.kappa}")
    # ---- inputs resident in HBM ----
    fp32 = Runner(prob, "fp32_ir", nbox, a.chunk, a.ir_max_iter, a.ir_tol, a.streams)
    for kv in a.tune:
        k, v = kv.split("=")
        fp32.plan.hps_plan_set_tuning(k, int(v))
    from paper_2503_04033_amd.solver import TwoLevelSolver  # noqa: F401  (import check of the package)
    i = fp32.info
    xi = torch.empty(nbox * i.n_i * 3, dtype=torch.float64, device=dev)
    xb = torch.empty(nbox * i.n_b * 3, dtype=torch.float64, device=dev)
    org = torch.tensor(prob.box_origins()[:nbox], device=dev)
    fp32.plan.hps_leaf_nodes(nbox, org, xi, xb)
    xi_h = xi.view(nbox, i.n_i, 3).cpu().numpy()
    xb_h = xb.view(nbox, i.n_b, 3).cpu().numpy()
    from paper_2503_04033_amd import interface as itf
    bmask = itf.boundary_mask(fp32.layout)[:nbox]
    b = torch.tensor(prob.b(xi_h), device=dev).contiguous()
    g_dir = torch.tensor(np.where(bmask, prob.g(xb_h), 0.0), device=dev).contiguous()
    torch.cuda.synchronize()
    # ---- FP32 + IR (headline) ----
    for _ in range(a.warmup):
        fp32.step(b, g_dir)
    torch.cuda.synchronize()
    fp32.ev = {k: [] for k in fp32.ev}
    fp32.plan.profile_enable(True)
    t0 = time.perf_counter()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(a.steps):
        fp32.step(b, g_dir, record=True)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1) / a.steps
    boxes_s = nbox / (ms / 1e3)
    phases = fp32.phase_ms()
    iters = fp32.iters.cpu().numpy()
    berr = fp32.berr.cpu().numpy()
    info_bad = int((fp32.infov.cpu().numpy() != 0).sum())
    log(f"fp32_ir: {ms:.1f} ms/step, {boxes_s:.1f} boxes/s (wall {wall:.1f} s); phases {phases}")
    steps = np.where(iters >= 0, iters, -1 - iters)  # corrections applied per box
    fams = fp32.plan.profile_read()
    # algorithmic flops per step: LU 2/3 n_i^3 per box; each solve pass 2 n_i^2 (n_b + 1) per
    # box that runs it (the library counts n_i^2 (n_b + 1) per sweep and active box)
    lu_alg = nbox * 2.0 / 3.0 * i.n_i ** 3
    solve_alg = (fams["solve_fwd"]["flops"] + fams["solve_bwd"]["flops"]) / a.steps
    solve_exec = (fams["solve_fwd"]["exec_flops"] + fams["solve_bwd"]["exec_flops"]) / a.steps
    tot_flops = lu_alg + solve_alg
    KNAMES = {"solve_fwd": "trsm_row128_kernel<float, false, false, 4>", "solve_bwd": "trsm_row128_kernel<float, true, false, 4>",
              "lu_gemm": "gemm_op_kernel<float, true>", "lu_panel": "lu_panel_kernel<float, 3, 16, 64, 1024>",
              "residual": "residual_mfma_kernel<14, 2, 4, double, false>"}
    # the LU/TRSM phase: device time of the factorization and solve kernels (events around
    # each launch) against the LU and solve flops of the step, algorithmic and as executed
    # (the first forward sweep skips the structurally zero leading rows of A_ib's columns)
    ph_ms = sum(fams[k]["ms"] for k in ("lu_gemm", "lu_panel", "lu_leaf", "solve_fwd", "solve_bwd")) / a.steps
    lu_trsm = {"ms_per_step": round(ph_ms, 3),
               "tflops": round(tot_flops / (ph_ms / 1e3) / 1e12, 2),
               "frac_fp32_mfma_peak": round(tot_flops / (ph_ms / 1e3) / PEAK_FP32_MFMA, 4),
               "tflops_executed": round((lu_alg + solve_exec) / (ph_ms / 1e3) / 1e12, 2),
               "frac_fp32_mfma_peak_executed": round((lu_alg + solve_exec) / (ph_ms / 1e3) / PEAK_FP32_MFMA, 4),
               "solve_flops_per_step": {"algorithmic": solve_alg, "executed": solve_exec},
               "first_forward_skipped_frac": None}
    fw = fams["solve_fwd"]
    if fw["flops"]:
        # executed / algorithmic of all forward sweeps; the first sweep is the one that skips
        first_alg = nbox * i.n_i ** 2 * (i.n_b + 1) * a.steps
        pad = (i.n_pad / i.n_i) ** 2
        lu_trsm["first_forward_skipped_frac"] = round(1.0 - (fw["exec_flops"] - (fw["flops"] - first_alg) * pad) /
                                                      (first_alg * pad), 4)
    dom = max(fams, key=lambda k: fams[k]["ms"])
    fd = fams[dom]
    achieved = fd["flops"] / (fd["ms"] / 1e3) if fd["ms"] > 0 else 0.0
    # bandwidth kernels: algorithmic HBM bytes per step over their event time
    nrhs = i.n_b + 1
    # first pass: FP32 X read, R32 written (8 bytes per entry); after each correction a
    # check pass reads the FP64 X (8); a box that takes another correction forms R32
    # again (12: FP64 X read, R32 written)
    res_bytes = (nbox * i.n_i * nrhs * 8.0 + float(steps.sum()) * i.n_i * nrhs * 8.0
                 + float(np.maximum(steps - 1, 0).sum()) * i.n_i * nrhs * 12.0)
    bw = {"operators": nbox * (i.n_pad ** 2 * 4.0 + i.n_i * 8.0),
          "dtn": nbox * (i.n_i * nrhs * 8.0 + i.n_b ** 2 * 8.0 + i.n_b * 8.0),
          "residual": res_bytes}
    bandwidth = {}
    for k, byt in bw.items():
        t = fams[k]["ms"] / a.steps / 1e3
        if t > 0:
            bandwidth[k] = {"ms_per_step": round(t * 1e3, 3), "algorithmic_GB_per_step": round(byt / 1e9, 3),
                            "TB_s": round(byt / t / 1e12, 3), "frac_hbm_peak": round(byt / t / PEAK_HBM, 4)}
    result = {
        "metric": METRIC, "value": round(boxes_s, 2), "unit": "boxes/s", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32 MFMA LU/solves + f64 refinement and DtN", "data": "synthetic",
        "config": {"workload": "16x16x16 leaf boxes, p=16 (2744 interior nodes/box), kappa=40, "
                               "b=1+0.3*sum of 8 seeded Gaussian bumps (width 0.1), plane-wave g, f=0",
                   "nbox": nbox, "p": prob.p, "n_i": i.n_i, "n_b": i.n_b, "chunk": fp32.chunk, "streams": a.streams,
                   "ir_tol": a.ir_tol, "ir_max_iter": a.ir_max_iter},
        "mfma_frac_lu_solve": round(tot_flops / (ms / 1e3) / PEAK_FP32_MFMA, 4),
        "tflops_lu_solve": round(tot_flops / (ms / 1e3) / 1e12, 2),
        "lu_trsm_phase": lu_trsm,
        "ir": {"iters_hist": {int(k): int(v) for k, v in zip(*np.unique(iters, return_counts=True))},
               "berr_max": float(berr.max()), "lu_info_nonzero": info_bad},
        "phase_ms_per_step": {k: round(v["ms_total"] / a.steps, 3) for k, v in phases.items()},
        "kernel_families_per_step": {k: {"launches": v["launches"] // a.steps, "ms": round(v["ms"] / a.steps, 3),
                                         "tflops": round(v["flops"] / (v["ms"] / 1e3) / 1e12, 2) if v["ms"] and v["flops"] else None,
                                         "tflops_executed": round(v["exec_flops"] / (v["ms"] / 1e3) / 1e12, 2) if v["ms"] and v["exec_flops"] else None}
                                     for k, v in fams.items()},
        "bandwidth_kernels": bandwidth,
        "roofline": {"kernel": KNAMES.get(dom, dom), "bound": "mfma" if fd["flops"] else "hbm",
                     "achieved": round(achieved / 1e12, 3), "peak": PEAK_FP32_MFMA / 1e12, "unit": "TFLOP/s",
                     "frac": round(achieved / PEAK_FP32_MFMA, 4), "traffic": measured_traffic(KNAMES.get(dom, dom)),
                     "per_launch": {"launches": fd["launches"], "avg_ms": round(fd["ms"] / max(fd["launches"], 1), 4),
                                    "avg_algorithmic_flops": fd["flops"] / max(fd["launches"], 1),
                                    "avg_executed_flops": fd["exec_flops"] / max(fd["launches"], 1)}},
    }
    log(f"whole path {tot_flops / (ms / 1e3) / 1e12:.2f} TFLOP/s; dominant {dom}: {achieved / 1e12:.2f} TFLOP/s")
    # ---- FP64 path beside it ----
    if not a.no_fp64:
        T32 = fp32.T_vals.clone()
        g32 = fp32.g_loads.clone()
        del fp32
        torch.cuda.empty_cache()
        # FP64 buffers are ~1.4x larger per box: the same streams, chunks of chunk/streams
        fp64 = Runner(prob, "fp64", nbox, max(1, min(a.chunk, 1024) // a.streams), streams=a.streams)
        fp64.step(b, g_dir)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fp64.step(b, g_dir, record=True)
        e1.record()
        torch.cuda.synchronize()
        ms64 = e0.elapsed_time(e1)
        dT = float(torch.linalg.norm(T32 - fp64.T_vals) / torch.linalg.norm(fp64.T_vals))
        dg = float(torch.linalg.norm(g32 - fp64.g_loads) / torch.linalg.norm(fp64.g_loads))
        result["fp64_path"] = {"boxes_per_s": round(nbox / (ms64 / 1e3), 2), "ms_per_step": round(ms64, 3),
                               "chunk": fp64.chunk, "streams": a.streams,
                               "speedup_fp32ir_over_fp64": round(ms64 / ms, 3),
                               "rel_err_T_fp32ir_vs_fp64": dT, "rel_err_g_fp32ir_vs_fp64": dg,
                               "phase_ms": {k: round(v["ms_total"], 3) for k, v in fp64.phase_ms().items()}}
        log(f"fp64: {ms64:.1f} ms/step; dT {dT:.2e} dg {dg:.2e}")
        del fp64
        torch.cuda.empty_cache()
    if not a.no_solve_stage and not a.nbox:
        # end to end (build, interface factorization and solve, interiors) where the host
        # interface solve fits: the same family at 4x4x4 boxes, p = 16, kappa = 40
        small = W.multi_bump((4, 4, 4), 16, 40.0, 3, name="cfg3_4x4x4_p16")
        legs = {}
        for prec, itf_kind in (("fp32_ir", "gpu"), ("fp64", "gpu"), ("fp64", "host")):
            key = f"{prec}_{itf_kind}"
            legs[key] = solve_stage(torch, small, prec, itf_kind)
            torch.cuda.empty_cache()
            log(f"solve stage {key}: { {k: v for k, v in legs[key].items() if k not in ('u_i', 'u_face')} }")
        ref = legs["fp64_host"]
        du = {k: float(torch.linalg.norm(v["u_i"] - ref["u_i"]) / torch.linalg.norm(ref["u_i"]))
              for k, v in legs.items() if k != "fp64_host"}
        df = {k: float(np.linalg.norm(v["u_face"] - ref["u_face"]) / np.linalg.norm(ref["u_face"]))
              for k, v in legs.items() if k != "fp64_host"}
        for v in legs.values():
            v.pop("u_i")
            v.pop("u_face")
        result["solve_stage_4x4x4_p16"] = {"legs": legs, "rel_diff_u_i_vs_fp64_host": du,
                                           "rel_diff_u_face_vs_fp64_host": df}
    if not a.no_solve_stage and not a.nbox:
        # time stepping with one build: diffusion-reaction on 4x4x4 boxes, p = 16
        pp = W.diffusion_reaction((4, 4, 4), 16, nu=0.05, dt=0.01, kappa=1.0, seed=9, width2=0.02)
        ts = {}
        for prec in ("fp32_ir", "fp64"):
            ts[prec] = time_stepping(torch, pp, prec, 10)
            torch.cuda.empty_cache()
            log(f"crank-nicolson {prec}: {ts[prec]}")
        result["crank_nicolson_4x4x4_p16"] = ts
        result["batch_config4"] = batch_config4(torch)
        log(f"config 4 batch: {result['batch_config4']}")
        result["adjoint_8x8x8_p10"] = adjoint_timing(torch)
        torch.cuda.empty_cache()
        log(f"adjoint: {result['adjoint_8x8x8_p10']}")
    if not a.no_cpu:
        result["cpu_baseline"] = cpu_baseline(prob, a.cpu_sample)
        log(f"cpu baseline {result['cpu_baseline']}")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
