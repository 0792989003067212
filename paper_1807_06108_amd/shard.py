"""Sample sharding of one controller: the exchange of the multi-GPU design,
carried out on one GPU with the host as the all-reduce.

Shard g holds samples [k_g, k_g + K_g) of the controller's sample set (its
configuration's sample_offset), so its draws are those of the unsharded
controller.  One iteration of every shard from the same U gives, per shard,
the statistics (rho_g = min S, eta_g = sum exp(-(S_k - rho_g)/lambda)) and
its own update U_g' = U + alpha dU_g / eta_g.  The unsharded update follows
by the log-sum-exp rescale of eq. (37):

    rho = min_g rho_g,  c_g = eta_g exp(-(rho_g - rho)/lambda),
    U' = U + sum_g c_g (U_g' - U) / sum_g c_g,

which is what a MIN all-reduce of rho and a SUM all-reduce of the rescaled
(eta_g, dU_g) would compute across GPUs (T*m + 2 numbers per shard).
"""

import math

import numpy as np
import torch

from .controller import Controller


def combine_updates(U, shard_U, shard_rho, shard_eta, shard_ok, lam):
    """The unsharded updated sequence from per-shard updates (fp64)."""
    U = np.asarray(U, dtype=np.float64)
    live = [g for g, ok in enumerate(shard_ok) if ok]
    if not live:
        return U.copy()
    rho = min(shard_rho[g] for g in live)
    c = {g: shard_eta[g] * math.exp(-(shard_rho[g] - rho) / lam) for g in live}
    tot = sum(c.values())
    out = U.copy()
    for g in live:
        out += (c[g] / tot) * (np.asarray(shard_U[g], dtype=np.float64) - U)
    return out


class ShardedController:
    """One controller's K samples split into shards, each run as its own
    launch; the shards' updates are combined on the host after every
    iteration and the combined sequence is given back to every shard."""

    def __init__(self, cfg, shards, U0=None):
        K = int(cfg["K"])
        bounds = np.linspace(0, K, shards + 1).astype(int)
        self.cfg = dict(cfg)
        self.lam = float(np.float32(cfg["lambda"]))
        self.parts = [Controller(dict(cfg, K=int(b - a), sample_offset=int(a)), U0)
                      for a, b in zip(bounds[:-1], bounds[1:])]
        self.U = self.parts[0].U.cpu().numpy().astype(np.float64)

    def step(self, x0, iters=1):
        """iters iterations from state x0; returns U (fp64 copy)."""
        for _ in range(iters):
            for c in self.parts:
                c.step(x0, 1)
            torch.cuda.synchronize()
            st = [c.stats() for c in self.parts]
            Ug = [c.U.cpu().numpy() for c in self.parts]
            self.U = combine_updates(self.U, Ug, [s["rho"] for s in st], [s["eta"] for s in st],
                                     [s["status"] == 0 for s in st], self.lam)
            U32 = self.U.astype(np.float32)
            for c in self.parts:
                c.set_U(U32)
            self.U = U32.astype(np.float64)
        return self.U.copy()

    @property
    def S(self):
        return np.concatenate([c.S.cpu().numpy() for c in self.parts])
