"""hipGraph capture of repeated launch sequences.

A step of fixed shape (e.g. detection + precoding of a batch of frames into
preallocated outputs) is captured once on a side stream and replayed; the
replay submits all kernels with one call.  The library's kernels allocate
nothing and record no memset nodes, so they capture as plain kernel nodes.
Schedules are looked up at capture time and fixed in the graph.
"""
from __future__ import annotations


class StepGraph:
    """Capture ``fn`` (which must only launch work on the current stream into
    preallocated buffers) and replay it."""

    def __init__(self, fn, warmup: int = 2):
        import torch
        self.torch = torch
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            for _ in range(warmup):
                fn()
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            fn()
        torch.cuda.synchronize()

    def replay(self) -> None:
        self.graph.replay()
