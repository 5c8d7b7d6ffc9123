"""Learned (normalised / offset) Min-Sum: autograd wrapper, training loop and
evaluation.  Every numerical step (frame generation, forward, backward, Adam,
decoding) runs in the HIP kernels of libldpc; this module only sequences them.

The learned decoder multiplies the check message magnitude mu of iteration t
of a row of degree class c by alpha[t][c] and subtracts beta[t][c], clipped
at zero; plain Min-Sum is alpha = 1, beta = 0.
"""
from __future__ import annotations

import torch

from . import ldpc


class NMSLoss(torch.autograd.Function):
    """loss = NMSLoss.apply(alpha, beta, llr, graph, ckpt_every, workspace, target)

    Mean over frames and bits of sum_{t=1..T} softplus((2c - 1) s^(t)), T =
    alpha.shape[0].  Backward gives d loss / d alpha, d beta and d llr from the
    hand-written reverse sweep (recomputing every ckpt_every iterations from
    checkpoints kept in `workspace`)."""

    @staticmethod
    def forward(ctx, alpha, beta, llr, graph, ckpt_every, workspace, target=None):
        loss, _ = ldpc.nms_train_forward(graph, llr, alpha, beta, ckpt_every, workspace, target=target)
        ctx.graph, ctx.k, ctx.ws, ctx.target = graph, ckpt_every, workspace, target
        ctx.save_for_backward(alpha, beta, llr)
        return loss[0]

    @staticmethod
    def backward(ctx, grad_out):
        alpha, beta, llr = ctx.saved_tensors
        # the scale of the incoming gradient is applied on the device
        ga, gb, gl = ldpc.nms_train_backward(ctx.graph, llr, alpha, beta, ctx.k, ctx.ws, grad_loss=1.0,
                                             target=ctx.target, want_llr_grad=ctx.needs_input_grad[2])
        g = grad_out.to(torch.float32)
        return ga * g, gb * g, (gl * g if gl is not None else None), None, None, None, None


class NMSTrainer:
    """Trains alpha, beta (T x n_classes) on frames generated on the GPU:
    all-zero codewords over BPSK/AWGN with Eb/N0 drawn per frame from a range
    (Min-Sum is symmetric in the transmitted codeword, so the all-zero
    codeword suffices), Adam updates by the library kernel."""

    def __init__(self, graph: ldpc.Graph, T: int = 10, batch: int = 4096, ckpt_every: int = 2,
                 ebn0_range=(1.0, 3.0), rate: float | None = None, lr: float = 1e-2, seed: int = 1234,
                 alpha0: float = 1.0, beta0: float = 0.0):
        self.g = graph
        self.T, self.B, self.k = T, batch, ckpt_every
        self.ebn0 = tuple(ebn0_range)
        self.rate = rate if rate is not None else 1.0 - graph.m / graph.n
        self.lr, self.seed = lr, seed
        dev = graph.device
        C = len(graph.check_degrees)
        self.alpha = torch.full((T, C), float(alpha0), dtype=torch.float32, device=dev)
        self.beta = torch.full((T, C), float(beta0), dtype=torch.float32, device=dev)
        self.m1 = [torch.zeros_like(self.alpha), torch.zeros_like(self.beta)]
        self.m2 = [torch.zeros_like(self.alpha), torch.zeros_like(self.beta)]
        self.ws = torch.empty(ldpc.train_workspace_bytes(graph, batch, T, ckpt_every), dtype=torch.uint8,
                              device=dev)
        self.steps = 0
        self.history = []

    def step(self) -> torch.Tensor:
        self.steps += 1
        llr = ldpc.awgn_llr(self.B, self.g.n, self.rate, self.ebn0, self.seed * 1_000_003 + self.steps,
                            self.g.device)
        a = self.alpha.clone().requires_grad_(True)
        b = self.beta.clone().requires_grad_(True)
        loss = NMSLoss.apply(a, b, llr, self.g, self.k, self.ws)
        loss.backward()
        ldpc.adam_step(self.alpha, a.grad.contiguous(), self.m1[0], self.m2[0], self.lr, self.steps)
        ldpc.adam_step(self.beta, b.grad.contiguous(), self.m1[1], self.m2[1], self.lr, self.steps)
        self.history.append(loss.detach())
        return loss.detach()

    def train(self, steps: int, log_every: int = 0, log=print, time_budget: float | None = None):
        """Run `steps` Adam steps, or fewer if `time_budget` seconds run out
        first (checked every 10 steps)."""
        import time
        t0 = time.time()
        for s in range(steps):
            loss = self.step()
            if log_every and (s + 1) % log_every == 0:
                log(f"[nms] step {self.steps} loss {float(loss):.5f} ({time.time() - t0:.1f} s)")
            if time_budget is not None and (s + 1) % 10 == 0:
                torch.cuda.synchronize()
                if time.time() - t0 > time_budget:
                    log(f"[nms] time budget reached after {s + 1} steps")
                    break
        return self

    def state_dict(self):
        return {"alpha": self.alpha.cpu(), "beta": self.beta.cpu(), "m1a": self.m1[0].cpu(),
                "m1b": self.m1[1].cpu(), "m2a": self.m2[0].cpu(), "m2b": self.m2[1].cpu(),
                "steps": self.steps, "T": self.T}

    def load_state_dict(self, d):
        dev = self.g.device
        self.alpha.copy_(d["alpha"].to(dev))
        self.beta.copy_(d["beta"].to(dev))
        self.m1[0].copy_(d["m1a"].to(dev))
        self.m1[1].copy_(d["m1b"].to(dev))
        self.m2[0].copy_(d["m2a"].to(dev))
        self.m2[1].copy_(d["m2b"].to(dev))
        self.steps = int(d["steps"])


def frame_errors(graph: ldpc.Graph, llr: torch.Tensor, max_iter: int, alpha=None, beta=None, codewords=None):
    """Decode (plain, or learned when alpha/beta are given) and count frame
    errors against the transmitted codewords (all-zero when None).  Returns
    (frame errors, bit errors, mean iterations, bits, iters)."""
    if alpha is None:
        bits, _, iters, _ = ldpc.minsum_decode(graph, llr, max_iter, want_post=False)
    else:
        bits, _, iters, _ = ldpc.nms_decode(graph, llr, max_iter, alpha, beta, want_post=False)
    ref = torch.zeros_like(bits) if codewords is None else codewords.to(torch.uint8)
    err = bits != ref
    return int(err.any(dim=1).sum()), int(err.sum()), float(iters.float().mean()), bits, iters
