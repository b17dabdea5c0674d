"""hipGraph capture of a detection step (QR, detector, epilogues for every
SNR point), replayed instead of relaunching each kernel.

Every library call only enqueues on torch's current stream and allocates
nothing, so a step can be captured with torch.cuda.graph.  Counters that a
step accumulates are cleared inside the step with a fill kernel (torch's
zero_), never with a memset node.
"""
from __future__ import annotations

import torch


class CapturedStep:
    def __init__(self, step_fn, warmup: int = 1):
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            for _ in range(warmup):
                step_fn()
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            step_fn()
        torch.cuda.synchronize()

    def replay(self):
        self.graph.replay()
