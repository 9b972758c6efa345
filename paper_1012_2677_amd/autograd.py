"""Differentiation of the LJ hot path through torch.autograd.

`LJEnergy`   (U, F) = (potential energy, forces) of positions q, with
             gradients of any scalar of (U, F) with respect to q, eps, sigma.
             Backward: dL/dq = -gU F - H gF (H = Hessian of U, so dF/dq = -H),
             dL/dtheta = gU dU/dtheta + gF . dF/dtheta, all from the HIP adjoint
             kernels (md_hvp, md_param_grad).
`TrajectoryMeanPE`  O = (1/K) sum_{k=1..K} U(q_k) over K velocity-Verlet steps
             from (q0, v0), differentiated with respect to q0 (v0 held fixed),
             eps and sigma.  The forward pass stores (q, v) every `ckpt` steps;
             the backward pass recomputes each segment from its checkpoint and
             sweeps it in reverse (adjoint of velocity Verlet, below).

Positions are (N, 3) float64 CUDA tensors in a periodic box; the wrap into the
box is a relabelling of the same periodic point and is treated as the
identity by the derivatives.  Re-sorting is disabled here, so slots are the
caller's particle indices.
"""

from __future__ import annotations

import numpy as np
import torch

from . import _abi as A
from .engine import Engine, Grid, PairList, Workspace, make_params, stream_handle


class Field:
    """Grid, pair list and workspace for evaluating the force field and its
    adjoint at arbitrary positions of N particles (FP64, no re-sort)."""

    def __init__(self, n, box, eps, sigma, rc=2.5, rs=2.8, device="cuda"):
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.n = int(n)
        self.box, self.rc, self.rs = box, float(rc), float(rs)
        self.params = make_params(n, box, eps=float(eps), sigma=float(sigma), rc=rc, rs=rs,
                                  precision="fp64", resort_every=0)
        self.grid = Grid(self.params, self.device)
        self.plist = PairList(self.params, self.grid.ncell, self.device)
        self.ws = Workspace(self.params, self.device)
        self._own_pos = torch.empty((self.n, 4), dtype=torch.float64, device=self.device)
        self.pos = self._own_pos
        self.out2 = torch.empty(2, dtype=torch.float64, device=self.device)
        # the cell grid and list the passes use: the field's own, or those of
        # an engine whose last build was at the positions the field's would
        # have been built at (use_lists_of)
        self._cells, self._list = self.grid.c, self.plist.l
        # deferred list checks (defer_checks): the largest overflow flag of
        # the builds since the last check, on the device
        self.deferred = False
        self.overflow = torch.zeros(1, dtype=torch.int64, device=self.device)

    def set_params(self, eps, sigma):
        self.params.eps = float(eps)
        self.params.sigma = float(sigma)

    def set_positions(self, q: torch.Tensor, rebuild: bool = True):
        """Fold q into the box; bin it and build the pair list at rs unless
        rebuild is False (then the list of the previous call is kept, which is
        valid while no particle has moved more than (rs - rc)/2 since)."""
        q = q.detach().to(self.device, torch.float64).contiguous()
        st = stream_handle(self.device)
        self.pos = self._own_pos
        A.md_pack_positions(self.params, q.data_ptr(), self.pos.data_ptr(), st)
        if rebuild:
            self._build()

    def use_frame(self, frame: torch.Tensor, rebuild: bool = True):
        """Take a frame of positions already in the library's layout (N, 4),
        inside the box (a frame of md_step_record), without a copy; rebuild
        the pair list there unless rebuild is False."""
        assert frame.dtype == torch.float64 and frame.is_contiguous() and tuple(frame.shape) == (self.n, 4)
        self.pos = frame
        if rebuild:
            self._build()

    def use_lists_of(self, engine: Engine, frame: torch.Tensor):
        """Positions `frame` (as use_frame) with the cell grid and slot-entry
        pair list of `engine`, whose last build was at positions that every
        pair within rc of `frame` was listed at (its list is still valid
        there): no build.  The engine must not re-sort (slots = particles) and
        must not move on while the field uses its lists."""
        assert frame.dtype == torch.float64 and frame.is_contiguous() and tuple(frame.shape) == (self.n, 4)
        assert engine.n == self.n and int(engine.params.resort_every) == 0 and not engine.state.list.tiled
        self.pos = frame
        self._cells, self._list = engine.state.cells, engine.state.list

    def defer_checks(self, on: bool = True):
        """When on, a build does not wait to read its overflow flag: the flag
        is folded into `overflow` on the device, for check_lists() to read once
        for many builds (a list that overflowed has rows cut short, so every
        pass since must be redone after the list has grown)."""
        self.deferred = on
        self.overflow.zero_()

    def check_lists(self) -> bool:
        """True when no build overflowed since the last check (waits for the
        stream); otherwise grows the field's list for the next builds."""
        over = int(self.overflow.item())
        self.overflow.zero_()
        if over == 0:
            return True
        self.plist.grow_for(max(2 * int(self.plist.cell_stride), int(self.plist.status[1].item())))
        return False

    def _build(self):
        self._cells, self._list = self.grid.c, self.plist.l
        st = stream_handle(self.device)
        A.md_bin_cells(self.params, self.pos.data_ptr(), self.grid.c, self.ws.ptr, self.ws.nbytes, st)
        if self.deferred:
            A.md_build_pairlist(self.params, self.pos.data_ptr(), self.grid.c, self.plist.l, self.ws.ptr,
                                self.ws.nbytes, st)
            torch.maximum(self.overflow, self.plist.status[2:3], out=self.overflow)
            return
        for _ in range(4):
            A.md_build_pairlist(self.params, self.pos.data_ptr(), self.grid.c, self.plist.l, self.ws.ptr,
                                self.ws.nbytes, st)
            status = self.plist.status.cpu()
            if int(status[2]) == 0:
                return
            self.plist.grow_for(int(status[1]))
        raise A.MdError(A.MD_ERR_CAPACITY, "Field.set_positions", "pair list did not fit")

    def energy_forces(self):
        """(U, W, F[N, 3]) at the current positions."""
        F = torch.empty((3, self.n), dtype=torch.float64, device=self.device)
        A.md_forces(self.params, self.pos.data_ptr(), self._cells, self._list, F.data_ptr(),
                    self.out2.data_ptr(), self.ws.ptr, self.ws.nbytes, stream_handle(self.device))
        pw = self.out2.clone()
        return pw[0], pw[1], F.t()

    def hvp(self, u: torch.Tensor):
        """(H u [N, 3], u . dF/d(eps, sigma) [2]) at the current positions."""
        ut = u.detach().to(self.device, torch.float64).t().contiguous()
        Hu = torch.empty_like(ut)
        A.md_hvp(self.params, self.pos.data_ptr(), self._cells, self._list, ut.data_ptr(), Hu.data_ptr(),
                 self.out2.data_ptr(), self.ws.ptr, self.ws.nbytes, stream_handle(self.device))
        return Hu.t(), self.out2.clone()

    def adjoint_kick(self, u: torch.Tensor, out: torch.Tensor, u_out, coef, acc: torch.Tensor):
        """out = a out + b H u + c F;  acc += cu u.dF/dtheta + cU dU/dtheta;
        u_out = u + dt out (if given).  u, out, u_out: [3, N] float64."""
        A.md_adjoint_kick(self.params, self.pos.data_ptr(), self._cells, self._list, u.data_ptr(),
                          out.data_ptr(), None if u_out is None else u_out.data_ptr(), coef, acc.data_ptr(),
                          self.ws.ptr, self.ws.nbytes, stream_handle(self.device))

    def param_grad(self):
        """(dU/deps, dU/dsigma) at the current positions."""
        A.md_param_grad(self.params, self.pos.data_ptr(), self._cells, self._list, self.out2.data_ptr(),
                        self.ws.ptr, self.ws.nbytes, stream_handle(self.device))
        return self.out2.clone()


def _scalar(x) -> float:
    return float(x.detach().cpu()) if torch.is_tensor(x) else float(x)


class LJEnergy(torch.autograd.Function):
    """(U, F) = LJEnergy.apply(q, eps, sigma, box, rc=2.5, rs=2.8)."""

    @staticmethod
    def forward(ctx, q, eps, sigma, box, rc=2.5, rs=2.8):
        n = q.shape[0]
        f = Field(n, box, _scalar(eps), _scalar(sigma), rc, rs, q.device)
        f.set_positions(q)
        U, _, F = f.energy_forces()
        ctx.field = f
        ctx.save_for_backward(F)
        ctx.eps_like = eps if torch.is_tensor(eps) else None
        ctx.sig_like = sigma if torch.is_tensor(sigma) else None
        return U.to(q.dtype), F.contiguous()

    @staticmethod
    def backward(ctx, gU, gF):
        (F,) = ctx.saved_tensors
        f: Field = ctx.field
        n = F.shape[0]
        u = (gF if gF is not None else torch.zeros_like(F)).detach().to(torch.float64).t().contiguous()
        wU = 0.0 if gU is None else float(gU.detach().cpu())
        out = torch.empty((3, n), dtype=torch.float64, device=F.device)
        acc = torch.zeros(2, dtype=torch.float64, device=F.device)
        # dL/dq = -gU F - H gF;  dL/dtheta = gF . dF/dtheta + gU dU/dtheta
        f.adjoint_kick(u, out, None, (0.0, -1.0, -wU, 1.0, wU), acc)
        ge = acc[0].to(ctx.eps_like) if ctx.eps_like is not None else None
        gs = acc[1].to(ctx.sig_like) if ctx.sig_like is not None else None
        return out.t(), ge, gs, None, None, None


class TrajectoryMeanPE(torch.autograd.Function):
    """O = TrajectoryMeanPE.apply(q0, v0, eps, sigma, box, steps=200, ckpt=20,
    dt=0.005, rc=2.5, rs=2.8).

    Reverse sweep of one velocity-Verlet step (h = dt/2, unit mass, F = -grad U)
        v' = v + h F(q);  q' = q + dt v';  v'' = v' + h F(q')
    with adjoints (a_q, a_v) carried backwards:
        a_q  += -h H(q') a_v          (second kick)
        a_v  +=  dt a_q               (drift)
        a_q  += -h H(q) a_v           (first kick)
    and the observable adds (1/K) grad U(q') = -(1/K) F(q') to a_q at every
    step; the parameter adjoint gathers h a_v . dF/dtheta at both kicks and
    (1/K) dU/dtheta at every sampled state.  The first kick of step k and the
    second kick of step k - 1 both act at q_k with the same a_v, so every
    state but q_0 and q_K takes one fused adjoint pass (coefficient 2h).
    """

    @staticmethod
    def forward(ctx, q0, v0, eps, sigma, box, steps=200, ckpt=20, dt=0.005, rc=2.5, rs=2.8):
        e_, s_ = _scalar(eps), _scalar(sigma)
        dev = q0.device
        q = q0.detach().to(torch.float64)
        v = v0.detach().to(torch.float64)
        ckpts = []
        total = 0.0
        k = 0
        eng = Engine(q.cpu().numpy(), v.cpu().numpy(), box, eps=e_, sigma=s_, rc=rc, rs=rs, dt=dt,
                     precision="fp64", resort_every=0, device=dev)
        while k < steps:
            ckpts.append((eng.pos[:, :3].clone(), eng.vel.t().clone()))
            m = min(ckpt, steps - k)
            log = eng.step(m, sample_every=1)
            total += float(np.sum(log[:, 1]))
            k += m
        ctx.ckpts = ckpts
        ctx.cfg = dict(box=box, steps=steps, ckpt=ckpt, dt=dt, rc=rc, rs=rs, eps=e_, sigma=s_)
        ctx.eps_like = eps if torch.is_tensor(eps) else None
        ctx.sig_like = sigma if torch.is_tensor(sigma) else None
        return torch.tensor(total / steps, dtype=torch.float64, device=dev)

    @staticmethod
    def backward(ctx, gO):
        cfg = ctx.cfg
        K, dt = cfg["steps"], cfg["dt"]
        h = 0.5 * dt
        q0, _ = ctx.ckpts[0]
        dev = q0.device
        n = q0.shape[0]
        f = Field(n, cfg["box"], cfg["eps"], cfg["sigma"], cfg["rc"], cfg["rs"], dev)
        f.params.dt = dt
        w = float(gO.detach().cpu()) / K
        aq = torch.zeros((3, n), dtype=torch.float64, device=dev)
        av = torch.zeros_like(aq)
        av_next = torch.empty_like(aq)
        acc = torch.zeros(2, dtype=torch.float64, device=dev)
        # pair lists: the recomputation of a segment rebuilds its list by the
        # rule of every run (some particle moved more than (rs - rc)/2 since the
        # last build), so a list built at one of the states it rebuilt at holds
        # every pair within rc up to the next such state; the reverse sweep
        # builds its lists at those states only
        k_end = K
        # one engine recomputes every segment, reset from each checkpoint
        eng = Engine(np.zeros((n, 3)), np.zeros((n, 3)), cfg["box"], eps=cfg["eps"], sigma=cfg["sigma"],
                     rc=cfg["rc"], rs=cfg["rs"], dt=dt, precision="fp64", resort_every=0, device=dev)
        # the field's list builds do not wait for their overflow flags: the
        # flags are read once per segment, and a segment whose list overflowed
        # is swept again from its saved adjoints with a grown list
        f.defer_checks(True)
        for si in range(len(ctx.ckpts) - 1, -1, -1):
            qc, vc = ctx.ckpts[si]
            k0 = si * cfg["ckpt"]
            m = k_end - k0
            # recompute the segment's states q_k0 .. q_k0+m from its checkpoint
            # in one run that records them (state t >= 1 is frame t - 1)
            eng.reset(qc, vc)
            eng.prepare()                 # the list of state 0
            frame0 = eng.pos.clone()      # state 0 in the library's layout (the prepared positions)
            _, frames, built = eng.step_record(m)
            builds = [0] + [t + 1 for t in range(m) if built[t]]   # states the segment's lists were built at
            saved = (aq.clone(), av.clone(), acc.clone())
            while True:
                av, av_next = _sweep_segment(f, eng, frame0, frames, builds, aq, av, av_next, acc, k0, m, k_end,
                                             K, h, w)
                if f.check_lists():
                    break
                aq.copy_(saved[0])
                av.copy_(saved[1])
                acc.copy_(saved[2])
            k_end = k0
        ge = acc[0].to(ctx.eps_like) if ctx.eps_like is not None else None
        gs = acc[1].to(ctx.sig_like) if ctx.sig_like is not None else None
        return aq.t(), None, ge, gs, None, None, None, None, None, None


def _sweep_segment(f, eng, frame0, frames, builds, aq, av, av_next, acc, k0, m, k_end, K, h, w):
    """Reverse sweep of one recomputed segment (states k0 .. k0 + m), updating
    aq and acc in place and av through the two velocity-adjoint buffers;
    returns (av, av_next), the buffer then holding av first.  The states
    from the segment's last build on use the recomputing engine's own list
    (built there, still valid: the engine stands at the segment's end), the
    earlier ones the field's list built at the same states."""
    current = None                # build state of the field's own list
    last = builds[-1]

    def place(t):
        nonlocal current
        frame = frame0 if t == 0 else frames[t - 1]
        b = max(x for x in builds if x <= t)
        if b == last:
            f.use_lists_of(eng, frame)
            return
        if b != current:
            f.use_frame(frame0 if b == 0 else frames[b - 1])
            current = b
        f.use_frame(frame, rebuild=False)


    # states k = k0 + t, from the segment's top down to k0 (the top state
    # k_end was taken by the later segment unless it is q_K)
    t_top = m if k_end == K else m - 1
    for t in range(t_top, -1, -1):
        k = k0 + t
        place(t)
        if k == K:
            # second kick of the last step and the observable term at q_K,
            # with the drift of the velocity adjoint fused in
            f.adjoint_kick(av, aq, av_next, (1.0, -h, -w, h, w), acc)
            av, av_next = av_next, av
        elif k > 0:
            # the first kick of step k and the second kick of step k - 1 act
            # at the same q_k with the same velocity adjoint: one pass with
            # both (2h), the observable term, and the drift
            f.adjoint_kick(av, aq, av_next, (1.0, -2.0 * h, -w, 2.0 * h, w), acc)
            av, av_next = av_next, av
        else:
            # first kick of step 0 at q_0
            f.adjoint_kick(av, aq, None, (1.0, -h, 0.0, h, 0.0), acc)
    return av, av_next
