"""torch.autograd.Function over K-step KDK rollouts.

Forward: one force pass at x0 (nbody_forces) and `steps` KDK steps
(nbody_rollout) that write FP64 checkpoints of (x, v) every `ckpt_every` steps.
Backward: nbody_rollout_backward, the exact discrete adjoint of those steps,
recomputing the positions between checkpoints. Gradients flow to the initial
positions, velocities and the masses. With ckpt_every = 0 no checkpoints are kept:
the backward pass rebuilds the trajectory by integrating backwards from the final
state (nbody_rollout_backward_reversible; O(n) memory, exact up to rounding that
chaotic dynamics amplify).
"""
from __future__ import annotations

import torch


class NBodyRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, pos0, vel0, mass, dt, steps, ckpt_every, G, eps, precision, offsets):
        from . import forces, rollout
        pos = pos0.detach().clone().contiguous()
        vel = vel0.detach().clone().contiguous()
        m = mass.detach().contiguous()
        acc, _ = forces(pos, m, G=G, eps=eps, precision=precision, offsets=offsets)
        ckpt, _ = rollout(pos, vel, m, acc, dt, steps, ckpt_every=ckpt_every, G=G, eps=eps,
                          precision=precision, offsets=offsets)
        if ckpt_every == 0:
            ctx.save_for_backward(m, pos.clone(), vel.clone())
        else:
            ctx.save_for_backward(m, ckpt)
        ctx.args = (dt, steps, ckpt_every, G, eps, precision, offsets)
        return pos, vel

    @staticmethod
    def backward(ctx, gpos, gvel):
        from . import rollout_backward, rollout_backward_reversible
        saved = ctx.saved_tensors
        m = saved[0]
        dt, steps, ckpt_every, G, eps, precision, offsets = ctx.args
        if gpos is None:
            gpos = torch.zeros((3, m.shape[0]), dtype=torch.float64, device=m.device)
        if gvel is None:
            gvel = torch.zeros((3, m.shape[0]), dtype=torch.float64, device=m.device)
        if ckpt_every == 0:
            gx, gv, gm = rollout_backward_reversible(m, saved[1], saved[2], gpos.contiguous(), gvel.contiguous(), dt,
                                                     steps, G=G, eps=eps, precision=precision, offsets=offsets)
        else:
            gx, gv, gm = rollout_backward(m, saved[1], gpos.contiguous(), gvel.contiguous(), dt, steps, ckpt_every,
                                          G=G, eps=eps, precision=precision, offsets=offsets)
        return gx, gv, gm, None, None, None, None, None, None, None


def rollout_fn(pos0, vel0, mass, dt, steps, ckpt_every=None, *, G=1.0, eps=1e-2, precision="fp32c", offsets=None):
    """Differentiable rollout: returns (x_K, v_K); gradients w.r.t. pos0, vel0, mass.
    ckpt_every=None picks about sqrt(steps); 0 keeps no checkpoints (reversible backward)."""
    if ckpt_every is None:
        ckpt_every = max(1, int(round(steps ** 0.5)))
    if ckpt_every < 0:
        raise ValueError("ckpt_every must be >= 0")
    return NBodyRollout.apply(pos0, vel0, mass, float(dt), int(steps), int(ckpt_every), float(G), float(eps),
                              precision, offsets)
