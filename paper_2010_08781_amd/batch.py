"""The batched workload as one graph launch.

BatchPlan captures, into one hipGraph, a device-driven batched SSSP run
(up to 256 unit-weight sources on one graph, supersteps enqueued up to a
cap) followed by a PageRank run over a disjoint union of graphs with
per-part vertex counts.  A replay is a single graph launch with no host
synchronisation inside; the outcome is read afterwards.

    plan = BatchPlan(g22, sources, union, parts, updates=20)
    plan.capture()
    plan.replay()
    dist, stats = plan.sssp()          # [Q, N] distances, summed trace
    ranks = plan.ranks()               # PageRank of every part
"""
from __future__ import annotations

from typing import Optional

import paper_2010_08781_amd as ipg


class BatchPlan:
    def __init__(self, sssp_graph, sources, pr_graph, parts, updates: int = 20, max_supersteps: int = 64,
                 sssp_tuning: Optional[dict] = None, pr_tuning: Optional[dict] = None):
        import torch

        self.gs, self.gp = sssp_graph, pr_graph
        self.sources = torch.as_tensor(sources, dtype=torch.int64).to(torch.int32).to(sssp_graph.device)
        self.parts = parts
        self.updates = int(updates)
        self.max_supersteps = int(max_supersteps)
        self.sssp_tuning, self.pr_tuning = sssp_tuning, pr_tuning
        self.dist = torch.empty((self.sources.numel(), sssp_graph.n), dtype=torch.int32, device=sssp_graph.device)
        self.graph = None

    def _enqueue(self):
        self.gs.run_multi_sssp(self.sources, max_supersteps=self.max_supersteps, out=self.dist,
                               tuning=self.sssp_tuning, enqueue=True)
        self.gp.run("pagerank", self.updates, mode="pull", parts=self.parts, tuning=self.pr_tuning, enqueue=True)

    def run_eager(self):
        """The same work launched directly (no graph), then synchronised."""
        import torch

        self._enqueue()
        torch.cuda.synchronize()

    def capture(self):
        import torch

        self.run_eager()  # first use of the workspaces and the library's queries, outside the capture
        self.graph = torch.cuda.CUDAGraph()
        stream = torch.cuda.Stream()
        stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.graph(self.graph, stream=stream):
            self._enqueue()
        torch.cuda.current_stream().wait_stream(stream)
        torch.cuda.synchronize()
        return self

    def replay(self):
        self.graph.replay()

    def sssp(self):
        """(distances, RunStats) of the batched SSSP of the last replay or eager run."""
        return self.dist, self.gs.multi_sssp_result()

    def ranks(self):
        return self.gp.read_values(ipg.APP_PAGERANK)
