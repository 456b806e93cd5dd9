"""Training data and training loop for the interpolation-weight MLP (an
addition to the paper; see bamg_mlp_* in include/bamg.h).

The network learns what a second bootstrap cycle (BAMG^2, Section 7) does to
the first cycle's interpolation rows: for every F point of every level,
its input is the cycle-1 feature vector and its target is the correction
from the cycle-1 least-squares row (features 80..87) to the row the second
cycle produces. The setup then takes a one-cycle hierarchy with those
corrections applied where they pass the objective test (learned="use").
All arithmetic runs in the library's kernels; this module only gathers the
harvested tensors and calls the trainer.
"""
import numpy as np

from . import MLP, Hierarchy, mlp_init_params, options_for


def harvest(chains, **kw):
    """Features X and correction targets T with mask M from BAMG^2 setups of
    `chains` (each with the options in kw): CUDA float32 tensors."""
    import torch
    Xs, Ts, Ms = [], [], []
    for ch in chains:
        h = Hierarchy.from_chain(ch, options_for(ch, setup_cycles=2, learned="record", **kw))
        for l in range(h.levels - 1):
            X, T, M = h.harvest(l)
            Xs.append(X)
            Ts.append((T - X[:, 80:88]) * M)
            Ms.append(M)
        h.close()
    return torch.cat(Xs), torch.cat(Ts), torch.cat(Ms)


def train(X, T, M, seed=2024, epochs=120, batch=1024, lr=1e-3, lr_final=3e-4):
    """Train a fresh network (seeded initialisation and sample order): Adam
    at `lr` for `epochs` passes, then at `lr_final` for as many again.
    Returns the network and the per-epoch losses."""
    import torch
    perm = torch.from_numpy(np.random.default_rng(seed).permutation(X.shape[0])).to(X.device)
    X, T, M = X[perm].contiguous(), T[perm].contiguous(), M[perm].contiguous()
    net = MLP(mlp_init_params(seed))
    l1 = net.train(X, T, M, batch=batch, epochs=epochs, lr=lr)
    l2 = net.train(X, T, M, batch=batch, epochs=epochs, lr=lr_final)
    return net, np.concatenate([l1, l2])
