"""Gradients of a shock-profile misfit with respect to the relaxation times.

Forward: n_steps of the LB-SMRT step from a fixed initial state, with a
checkpoint of the state every `checkpoint_every` steps; the misfit
    L = sum_x [s_rho^2 (rho - rho*)^2 + s_theta^2 (theta - theta*)^2 + s_q^2 (q_x - q_x*)^2]
of the final pre-collision moments.  Backward: for each segment in reverse,
restore its checkpoint, replay it storing every state, then run the adjoint
step (lbsmrt_step_adjoint) backwards through it.  Every step of the forward
and reverse sweeps runs in the HIP library; this module only sequences calls
and holds device buffers.
"""
import torch

from .lattice import Lattice


def tau_keys(N):
    """Relaxation times that act, in a fixed order: (n, m), n = 2..N, (2,1) excluded."""
    return [(n, m) for n in range(2, N + 1) for m in range(n // 2 + 1) if (n, m) != (2, 1)]


class ShockFit:
    """Holds the lattice, the initial state, the target profiles and the buffers."""

    def __init__(self, lattice: Lattice, f0: torch.Tensor, target: torch.Tensor, scales, n_steps: int,
                 checkpoint_every: int = 100):
        if n_steps < 1 or checkpoint_every < 1:
            raise ValueError("n_steps and checkpoint_every must be positive")
        self.lat = lattice
        self.f0 = f0
        self.target = target.to(torch.float64).contiguous()
        if self.target.shape != (3, lattice.n_nodes):
            raise ValueError("target must be (3, n_nodes): rho*, theta*, q_x*")
        self.scales = [float(s) for s in scales]
        self.n_steps = int(n_steps)
        self.every = int(checkpoint_every)
        self.keys = tau_keys(lattice.N)
        n_seg = (self.n_steps + self.every - 1) // self.every
        self._ckpt = [lattice.new_state() for _ in range(n_seg)]
        self._seg = [lattice.new_state() for _ in range(min(self.every, self.n_steps) + 1)]
        self._lam = [lattice.new_state(), lattice.new_state()]
        self._fin = lattice.new_state()
        self._loss = torch.zeros(1, dtype=torch.float64, device=lattice.device)
        self._dtau = torch.zeros(18, dtype=torch.float64, device=lattice.device)
        self._final = None

    def set_tau(self, tau_vec):
        self.lat.set_tau({k: float(v) for k, v in zip(self.keys, tau_vec)})

    def forward(self):
        """Run the forward sweep, keep checkpoints, return L (float)."""
        lat = self.lat
        cur = self._seg[0]
        cur.copy_(self.f0)
        nxt = self._seg[1]
        for t in range(self.n_steps):
            if t % self.every == 0:
                self._ckpt[t // self.every].copy_(cur)
            lat.step(cur, nxt, 1)
            cur, nxt = nxt, cur
        self._fin.copy_(cur)
        self._final = self._fin
        lat.loss_seed(cur, self.target, self.scales, self._lam[0], self._loss)
        lat.sync()
        return float(self._loss.item())

    def backward(self):
        """dL/dtau in the order of self.keys (requires forward() first)."""
        lat = self.lat
        self._dtau.zero_()
        lam, lam_prev = self._lam
        lat.loss_seed(self._final, self.target, self.scales, lam, self._loss)
        n_seg = len(self._ckpt)
        for s in reversed(range(n_seg)):
            t0 = s * self.every
            n = min(self.every, self.n_steps - t0)
            self._seg[0].copy_(self._ckpt[s])
            for k in range(n - 1):
                lat.step(self._seg[k], self._seg[k + 1], 1)
            for k in reversed(range(n)):
                lat.step_adjoint(self._seg[k], lam, lam_prev, self._dtau)
                lam, lam_prev = lam_prev, lam
        lat.sync()
        self._lam_f0 = lam
        g = self._dtau.view(6, 3).cpu()
        return [float(g[n, m]) for (n, m) in self.keys]


class SMRTShockLoss(torch.autograd.Function):
    """L(tau) for a ShockFit; backward returns dL/dtau from the adjoint sweep."""

    @staticmethod
    def forward(ctx, tau_vec, fit):
        fit.set_tau(tau_vec.detach().cpu().tolist())
        L = fit.forward()
        ctx.fit = fit
        return torch.tensor(L, dtype=torch.float64)

    @staticmethod
    def backward(ctx, grad_out):
        g = ctx.fit.backward()
        return grad_out * torch.tensor(g, dtype=torch.float64), None
