"""Training driver of the learned (1,1)-diagonal correction.

Argument marshalling only: the seeded training elements are drawn on the host
(`inputs.training_elements`), and the library generates their targets
(hd_learned_targets: projected-gradient minimisation of the local pencil
spread, one workgroup per element), their features (hd_learned_features) and
trains the network (hd_mlp_train) on the GPU.  The trained network stays in
the context; `hd_build_precond` with learned = 1 then applies it to the mesh
(BF16 inference) before the diagonal, S~ and the AMG are built.
"""
import numpy as np

from . import inputs


def build_dataset(ctx, n, seed=50, max_steps=30, progress=None):
    """Features x [n, 27] (float32), targets theta* [n, 6] (float32) and
    the spreads (at 0, at theta*) [n, 2] of n seeded training elements.
    `progress(msg)`, if given, is called after each degree's targets."""
    import torch
    V, p, alpha, beta = inputs.training_elements(n, seed)
    dev = ctx.device
    theta = torch.empty((n, 6), dtype=torch.float64, device=dev)
    spread = torch.empty((n, 2), dtype=torch.float64, device=dev)
    for pp in range(1, 7):
        idx = np.nonzero(p == pp)[0]
        if len(idx) == 0:
            continue
        Vd = torch.from_numpy(np.ascontiguousarray(V[idx])).to(dev)
        th, _, spr = ctx.learned_targets(pp, Vd, max_steps)
        it = torch.from_numpy(idx).to(dev)
        theta[it] = th
        spread[it] = spr
        if progress:
            torch.cuda.synchronize(dev)
            progress(f'targets p={pp}: {len(idx)} elements')
    Vd = torch.from_numpy(np.ascontiguousarray(V)).to(dev)
    x = ctx.learned_features(Vd, torch.from_numpy(alpha).to(dev), torch.from_numpy(beta).to(dev),
                             torch.from_numpy(p.astype(np.int32)).to(dev))
    return x, theta.float().contiguous(), spread


def train(ctx, n=200000, seed=50, max_steps=30, epochs=20, batch=512, lr=1e-3, val_frac=0.1, progress=None):
    """Generate the data set, initialise the network from `seed` and train it;
    returns per-epoch training and validation losses and the data set's
    mean spread before and after the target scalings."""
    x, y, spread = build_dataset(ctx, n, seed, max_steps, progress)
    nv = int(round(val_frac * n))
    nt = n - nv
    ctx.mlp_init(seed)
    tl, vl = ctx.mlp_train(x[:nt].contiguous(), y[:nt].contiguous(), x[nt:].contiguous() if nv else None,
                           y[nt:].contiguous() if nv else None, epochs=epochs, batch=batch, lr=lr, seed=seed)
    s = spread.cpu().numpy()
    return dict(train_loss=tl, val_loss=vl, spread0=float(np.nanmean(s[:, 0])), spread_opt=float(np.nanmean(s[:, 1])),
                n_train=nt, n_val=nv)
