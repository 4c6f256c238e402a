"""Batched leaf reduction of several independent problems in one stream (spec a7).

The paper batches boxes of one polynomial order and suggests separate arrays per
order when p varies over a small set (Sec. 3.2, last paragraphs; its two-level
scheduler caps how many DtN maps are built at once).  Here every problem is a
size group with its own plan and buffers; each group is cut into chunks that
fit an HBM budget, and every chunk runs operators -> LU -> solves/refinement ->
DtN scatter as kernel launches that cover all boxes of the chunk.  The whole
sequence of launches can be captured once in a HIP graph and replayed (no host
work, no allocation, no memset nodes inside).  `autotune` picks, per group, the
chunk size and the plan's scheduling knobs (triangular-solve schedule and the
occupancy its kernels are built for) by timing candidates; none of these
choices changes a single bit of the results.
"""
from __future__ import annotations

import json
import os
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import torch

from . import interface as itf
from .leaf import LeafPlan, hps_interface_reduce
from .solver import _box_origins, fp64_redo


@dataclass
class Group:
    nboxes: tuple
    lo: tuple
    hi: tuple
    p: int
    kappa: float
    plan: LeafPlan = None
    layout: itf.InterfaceLayout = None
    chunk: int = 0
    bufs: dict = None
    b: torch.Tensor = None
    f: Optional[torch.Tensor] = None
    g_dir: torch.Tensor = None
    T_vals: torch.Tensor = None
    g_loads: torch.Tensor = None
    info: torch.Tensor = None
    iters: torch.Tensor = None
    berr: torch.Tensor = None
    slot_map: torch.Tensor = None
    triples: torch.Tensor = None
    extra: dict = field(default_factory=dict)

    @property
    def nbox(self) -> int:
        return int(np.prod(self.nboxes))

    @property
    def h(self):
        return tuple((self.hi[a] - self.lo[a]) / self.nboxes[a] for a in range(3))


def bytes_per_box(info) -> int:
    return info.a_bytes + info.perm_bytes + info.dinv_bytes + info.x_bytes + info.ws_bytes


class BatchedLeafReduction:
    """Build stage (Alg. 1 loop) for several problems, one stream, optional graph."""

    def __init__(self, problems, precision: str = "fp32_ir", hbm_budget: float = 64e9, ir_max_iter: int = 3,
                 ir_tol: Optional[float] = None, chunks: Optional[List[int]] = None, device="cuda",
                 tuning: Optional[List[dict]] = None):
        """chunks[q]: boxes per chunk of problem q (default: as many as fit hbm_budget).
        tuning[q]: plan knobs {name: value} for problem q (see LeafPlan.hps_plan_set_tuning)."""
        self.device = torch.device(device)
        self.precision = precision
        self.groups: List[Group] = []
        for q, pr in enumerate(problems):
            gr = Group(nboxes=tuple(pr.nboxes), lo=tuple(pr.lo), hi=tuple(pr.hi), p=int(pr.p), kappa=float(pr.kappa))
            gr.plan = LeafPlan(gr.p, gr.h, gr.kappa, precision, ir_max_iter, ir_tol)
            for k, v in ((tuning[q] if tuning else None) or {}).items():
                gr.plan.hps_plan_set_tuning(k, v)
            gr.layout = itf.build_layout(gr.nboxes, gr.plan.info.m)
            per_box = bytes_per_box(gr.plan.info)
            fit = max(1, int(hbm_budget // max(per_box, 1)))
            gr.chunk = int(chunks[q]) if chunks else min(gr.nbox, fit)
            self.groups.append(gr)
        self.graph = None

    def set_inputs(self, q: int, b: torch.Tensor, f: Optional[torch.Tensor], g_dir: torch.Tensor) -> None:
        gr = self.groups[q]
        gr.b, gr.f, gr.g_dir = b.contiguous(), (f.contiguous() if f is not None else None), g_dir.contiguous()

    def sample_inputs(self, q: int, prob) -> None:
        """Evaluate the problem's b, f, g at this group's nodes (device tensors)."""
        gr = self.groups[q]
        i = gr.plan.info
        org = torch.tensor(_box_origins(gr.nboxes, gr.lo, gr.h), device=self.device)
        xi = torch.empty(gr.nbox * i.n_i * 3, dtype=torch.float64, device=self.device)
        xb = torch.empty(gr.nbox * i.n_b * 3, dtype=torch.float64, device=self.device)
        gr.plan.hps_leaf_nodes(gr.nbox, org, xi, xb)
        xi_h = xi.view(gr.nbox, i.n_i, 3).cpu().numpy()
        xb_h = xb.view(gr.nbox, i.n_b, 3).cpu().numpy()
        bmask = itf.boundary_mask(gr.layout)
        b = torch.tensor(prob.b(xi_h), device=self.device)
        f = torch.tensor(prob.f(xi_h), device=self.device)
        g = torch.tensor(np.where(bmask, prob.g(xb_h), 0.0), device=self.device)
        gr.extra["xi"], gr.extra["xb"] = xi_h, xb_h
        self.set_inputs(q, b, f, g)

    def allocate(self) -> None:
        for gr in self.groups:
            i = gr.plan.info
            mm = i.m * i.m
            gr.bufs = gr.plan.alloc(gr.chunk, self.device)
            gr.T_vals = torch.zeros(gr.layout.nslot_total * mm * mm + 1, dtype=torch.float64, device=self.device)
            gr.g_loads = torch.zeros(gr.nbox, i.n_b, dtype=torch.float64, device=self.device)
            gr.info = torch.zeros(gr.nbox, dtype=torch.int32, device=self.device)
            gr.iters = torch.zeros(gr.nbox, dtype=torch.int32, device=self.device)
            gr.berr = torch.zeros(gr.nbox, dtype=torch.float64, device=self.device)
            gr.slot_map = torch.tensor(gr.layout.slot_map, device=self.device)
            gr.triples = torch.tensor(gr.layout.reduce_triples, device=self.device)

    @staticmethod
    def _enqueue_group(gr: Group) -> None:
        plan, B, C, mm = gr.plan, gr.bufs, gr.chunk, gr.plan.info.m ** 2
        for c0 in range(0, gr.nbox, C):
            nb = min(C, gr.nbox - c0)
            sl = slice(c0, c0 + nb)
            plan.hps_leaf_operators(nb, gr.b[sl], B["A"], B["anorm"])
            plan.hps_leaf_factor(nb, B["A"], B["perm"], B["dinv"], gr.info[sl])
            plan.hps_leaf_dtn(nb, B["A"], B["perm"], B["dinv"], gr.b[sl], B["anorm"],
                              gr.f[sl] if gr.f is not None else None, gr.g_dir[sl], gr.slot_map[sl],
                              gr.T_vals, gr.g_loads[sl], B["X"], gr.iters[sl], gr.berr[sl], B["ws"])
        if gr.triples.shape[0]:
            hps_interface_reduce(gr.triples, mm * mm, gr.T_vals)

    def enqueue(self, concurrent: bool = False) -> None:
        """All launches of the build stage for every group.  Sequential: one after another
        on the current stream.  Concurrent: each group on a stream of its own (default
        priority), forked from the current stream and joined back to it, so that the groups'
        kernels overlap (in a captured graph they become parallel branches); every group has
        its own plan and buffers, so the results are bitwise those of the sequential order."""
        if not concurrent or len(self.groups) < 2:
            for gr in self.groups:
                self._enqueue_group(gr)
            return
        main = torch.cuda.current_stream()
        if getattr(self, "_streams", None) is None:
            self._streams = [torch.cuda.Stream(device=self.device) for _ in self.groups]
        for st in self._streams:
            st.wait_stream(main)
        for gr, st in zip(self.groups, self._streams):
            with torch.cuda.stream(st):
                self._enqueue_group(gr)
        for st in self._streams:
            main.wait_stream(st)

    def capture(self, concurrent: bool = False) -> None:
        """Record the whole build stage in a HIP graph (after one eager warm-up run)."""
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.enqueue(concurrent)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self.enqueue(concurrent)
        torch.cuda.synchronize()

    def run(self, concurrent: bool = False) -> None:
        if self.graph is not None:
            self.graph.replay()
        else:
            self.enqueue(concurrent)

    def fallback(self) -> dict:
        """After run(): boxes whose FP64 refinement ended above ir_tol (ir_iters < 0) are
        factored and solved again with an FP64 plan, eagerly (outside any captured graph),
        and the shared diagonal blocks are reduced again (the reduction only reads the two
        boxes' own slots, so repeating it is exact).  Their ir_iters stay negative.
        Returns {group index: list of box ids redone}."""
        done = {}
        for q, gr in enumerate(self.groups):
            if self.precision != "fp32_ir":
                continue
            ids = torch.nonzero(gr.iters < 0).flatten().cpu().tolist()
            gr.extra["fp64_fallback"] = ids
            if not ids:
                continue
            if "plan64" not in gr.extra:
                gr.extra["plan64"] = LeafPlan(gr.p, gr.h, gr.kappa, "fp64")
            fp64_redo(gr.extra["plan64"], ids, gr.b, gr.f, gr.g_dir, gr.slot_map, gr.T_vals, gr.g_loads, gr.berr,
                      gr.chunk, self.device)
            if gr.triples.shape[0]:
                hps_interface_reduce(gr.triples, gr.plan.info.m ** 4, gr.T_vals)
            done[q] = ids
        return done


TRSM_KNOBS = ({"trsm_schedule": 0, "trsm_waves": 4}, {"trsm_schedule": 0, "trsm_waves": 6},
              {"trsm_schedule": 0, "trsm_waves": 8}, {"trsm_schedule": 1, "trsm_waves": 4})
RESIDUAL_KNOBS = ({"residual_cols": 8}, {"residual_cols": 4}, {"residual_cols": 2})
# the panel's thread count matters only where a 1024-thread panel exists (FP32 factors of
# 2049..3072 rows); the stage is skipped elsewhere
PANEL_KNOBS = ({"panel_threads": 1024}, {"panel_threads": 512})


def _panel_knob_applies(info, precision) -> bool:
    return precision == "fp32_ir" and 2048 < info.n_pad <= 3072


def _time_build(pr, precision, hbm_budget, chunk, knobs, reps):
    br = BatchedLeafReduction([pr], precision, hbm_budget, chunks=[chunk], tuning=[knobs])
    br.sample_inputs(0, pr)
    br.allocate()
    br.run()  # warm-up
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        br.run()
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del br
    torch.cuda.empty_cache()
    return ms


def autotune(problems, precision="fp32_ir", candidates=(128, 256, 512, 1024), hbm_budget=64e9, cache=None,
             reps=1, knob_stages=(TRSM_KNOBS, RESIDUAL_KNOBS, PANEL_KNOBS)):
    """Pick, per problem, the chunk size and the plan knobs by timing the build stage.

    One stage per group of knobs (solve schedule and occupancy, the residual's column
    blocking, the panel's thread count where it applies), each timed at the largest chunk
    that fits hbm_budget on top of the choices of the earlier stages; then every candidate
    chunk with the chosen knobs.
    Returns a list of {"chunk": c, "tuning": {knob: value}}; results are cached as JSON
    under the key (GPU name, p, nbox, precision).
    """
    name = torch.cuda.get_device_name(0)
    table = {}
    if cache and os.path.exists(cache):
        with open(cache) as fh:
            table = json.load(fh)
    out = []
    for pr in problems:
        nbox = int(np.prod(pr.nboxes))
        key = f"{name}|p={pr.p}|nbox={nbox}|{precision}"
        if key in table:
            out.append({"chunk": int(table[key]["chunk"]), "tuning": dict(table[key]["tuning"])})
            continue
        pinfo = LeafPlan(pr.p, pr.h, pr.kappa, precision).info
        per_box = bytes_per_box(pinfo)
        fits = [min(c, nbox) for c in candidates if per_box * min(c, nbox) <= hbm_budget]
        if not fits:
            raise ValueError(f"no candidate chunk of p={pr.p} fits {hbm_budget:.3g} bytes")
        c0 = max(fits)
        best_kn, ktrials = {}, []
        for stage in knob_stages:
            if stage is PANEL_KNOBS and not _panel_knob_applies(pinfo, precision):
                continue
            trials = [(dict(best_kn, **kn), _time_build(pr, precision, hbm_budget, c0, dict(best_kn, **kn), reps))
                      for kn in stage]
            best_kn = min(trials, key=lambda t: t[1])[0]
            ktrials += trials
        ctrials = {}
        for c in sorted(set(fits)):
            ctrials[c] = _time_build(pr, precision, hbm_budget, c, best_kn, reps)
        best_c = min(ctrials, key=ctrials.get)
        table[key] = {"chunk": best_c, "tuning": best_kn, "ms": ctrials[best_c],
                      "knob_trials": [[kn, ms] for kn, ms in ktrials],
                      "chunk_trials": {str(c): ms for c, ms in ctrials.items()}}
        out.append({"chunk": int(best_c), "tuning": dict(best_kn)})
    if cache:
        with open(cache, "w") as fh:
            json.dump(table, fh, indent=1)
    return out
