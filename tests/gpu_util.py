"""Test-side helpers that drive the C ABI on the GPU and decode its outputs.

Host logic only (decoding the documented list format); no method arithmetic.
"""

from __future__ import annotations

import numpy as np
import torch

SLOT_MASK = (1 << 27) - 1


def device():
    return torch.device("cuda", 0)


def to_pos4(q: np.ndarray) -> torch.Tensor:
    p4 = np.zeros((q.shape[0], 4))
    p4[:, :3] = q
    return torch.from_numpy(p4).to(device())


class Standalone:
    """Grid + pair list + workspace for standalone entry-point calls."""

    def __init__(self, q, L, *, rs=2.8, rc=2.5, eps=1.0, sigma=1.0, precision="fp64", cell_stride=None,
                 list_layout="auto"):
        from paper_1012_2677_amd import _abi as A
        from paper_1012_2677_amd.engine import Grid, PairList, Workspace, make_params, stream_handle

        self.A = A
        self.q = np.ascontiguousarray(q, dtype=np.float64)
        self.n = self.q.shape[0]
        self.params = make_params(self.n, L, eps=eps, sigma=sigma, rc=rc, rs=rs, precision=precision,
                                  resort_every=0, list_layout=list_layout)
        dev = device()
        self.grid = Grid(self.params, dev)
        self.plist = PairList(self.params, self.grid.ncell, dev, cell_stride)
        self.ws = Workspace(self.params, dev)
        self.pos = to_pos4(self.q)
        self.stream = stream_handle(dev)

    def bin(self):
        self.A.md_bin_cells(self.params, self.pos.data_ptr(), self.grid.c, self.ws.ptr, self.ws.nbytes, self.stream)
        torch.cuda.synchronize()
        return (self.grid.cell_of.cpu().numpy(), self.grid.count.cpu().numpy(), self.grid.start.cpu().numpy(),
                self.grid.order.cpu().numpy(), self.grid.cell_xyz.cpu().numpy())

    def build(self, grow=True):
        """Build the list; on overflow grow the cell stride and build again
        (unless grow=False).  Returns the status array."""
        for _ in range(3):
            self.A.md_build_pairlist(self.params, self.pos.data_ptr(), self.grid.c, self.plist.l, self.ws.ptr,
                                     self.ws.nbytes, self.stream)
            torch.cuda.synchronize()
            status = self.plist.status.cpu().numpy()
            if status[2] == 0 or not grow:
                return status
            self.plist.grow_for(int(status[1]))
        return status

    def forces(self, energy=True):
        dt = torch.float32 if self.params.precision == self.A.MD_MIXED else torch.float64
        F = torch.zeros((3, self.n), dtype=dt, device=device())
        pw = torch.zeros(2, dtype=torch.float64, device=device())
        self.A.md_forces(self.params, self.pos.data_ptr(), self.grid.c, self.plist.l, F.data_ptr(),
                         pw.data_ptr() if energy else None, self.ws.ptr, self.ws.nbytes, self.stream)
        torch.cuda.synchronize()
        return F.double().cpu().numpy().T.copy(), pw.cpu().numpy()

    def hvp(self, u):
        ut = torch.from_numpy(np.ascontiguousarray(u.T)).to(device())
        Hu = torch.zeros_like(ut)
        dp = torch.zeros(2, dtype=torch.float64, device=device())
        self.A.md_hvp(self.params, self.pos.data_ptr(), self.grid.c, self.plist.l, ut.data_ptr(), Hu.data_ptr(),
                      dp.data_ptr(), self.ws.ptr, self.ws.nbytes, self.stream)
        torch.cuda.synchronize()
        return Hu.cpu().numpy().T.copy(), dp.cpu().numpy()

    def adjoint_kick(self, u, out0, coef, with_u_out=True):
        """md_adjoint_kick with u, out0 given as (n, 3) arrays: returns
        (out, u_out or None, acc) with acc starting from zero."""
        ut = torch.from_numpy(np.ascontiguousarray(u.T)).to(device())
        out = torch.from_numpy(np.ascontiguousarray(out0.T)).to(device())
        u_out = torch.empty_like(ut) if with_u_out else None
        acc = torch.zeros(2, dtype=torch.float64, device=device())
        self.A.md_adjoint_kick(self.params, self.pos.data_ptr(), self.grid.c, self.plist.l, ut.data_ptr(),
                               out.data_ptr(), None if u_out is None else u_out.data_ptr(), tuple(coef),
                               acc.data_ptr(), self.ws.ptr, self.ws.nbytes, self.stream)
        torch.cuda.synchronize()
        uo = None if u_out is None else u_out.cpu().numpy().T.copy()
        return out.cpu().numpy().T.copy(), uo, acc.cpu().numpy()

    def param_grad(self):
        dU = torch.zeros(2, dtype=torch.float64, device=device())
        self.A.md_param_grad(self.params, self.pos.data_ptr(), self.grid.c, self.plist.l, dU.data_ptr(),
                             self.ws.ptr, self.ws.nbytes, self.stream)
        torch.cuda.synchronize()
        return dU.cpu().numpy()


def decode_rows(offsets, counts, nbr):
    """(key slot, partner slot, stencil code) for every entry of a full list."""
    n = offsets.shape[0]
    counts = counts.astype(np.int64)
    keys = np.repeat(np.arange(n, dtype=np.int64), counts)
    starts = np.repeat(offsets.astype(np.int64), counts)
    within = np.arange(keys.shape[0], dtype=np.int64) - np.repeat(np.cumsum(counts) - counts, counts)
    ent = nbr.view(np.uint32)[starts + within].astype(np.int64)
    return keys, ent & SLOT_MASK, ent >> 27


def pair_set_from_rows(keys, partners, ids=None):
    """Unordered pairs (min id, max id) and a check that each appears twice."""
    a = keys if ids is None else ids[keys]
    b = partners if ids is None else ids[partners]
    lo = np.minimum(a, b)
    hi = np.maximum(a, b)
    code = lo * (1 << 32) + hi
    uniq, cnt = np.unique(code, return_counts=True)
    return uniq, cnt


def pair_codes(pairs):
    p = np.asarray(pairs, dtype=np.int64)
    return np.sort(np.minimum(p[:, 0], p[:, 1]) * (1 << 32) + np.maximum(p[:, 0], p[:, 1]))


def force_error(F, Fref, S):
    """max_i |F_i - Fref_i| / S_i with S_i the sum of pair-force magnitudes on i."""
    err = np.linalg.norm(F - Fref, axis=1)
    return float(np.max(err / np.maximum(S, 1e-300)))


def hvp_scale(q, L, u, pairs, eps=1.0, sigma=1.0):
    """Per-particle scale of (H u)_i for an element-wise tolerance:
    sum over the pairs within rc of h_ij |u_j - u_i|, with h_ij an upper bound
    on the norm of the pair's 3x3 Hessian block (max(|V''|, |g|) <= |V''| + |g|,
    bounded by the magnitudes of the r^-14 and r^-8 terms of the plain LJ
    derivatives plus a margin for the small truncation terms).  A tolerance
    scale, not a result: it only normalises the error."""
    q = np.asarray(q, np.float64)
    L = np.broadcast_to(np.asarray(L, np.float64), (3,))
    i, j = pairs[:, 0].astype(np.int64), pairs[:, 1].astype(np.int64)
    d = q[j] - q[i]
    d -= L * np.rint(d / L)
    r2 = np.einsum("ij,ij->i", d, d)
    s6 = (sigma * sigma / r2) ** 3
    h = 4.0 * eps * (168.0 * s6 * s6 + 48.0 * s6) / r2 + 0.1 * eps / (sigma * sigma)
    du = np.linalg.norm(np.asarray(u)[j] - np.asarray(u)[i], axis=1)
    out = np.zeros(q.shape[0])
    np.add.at(out, i, h * du)
    np.add.at(out, j, h * du)
    return out


def elementwise_error(X, Xref, scale):
    """max_i |X_i - Xref_i| / scale_i (rows of (n, 3) arrays)."""
    err = np.linalg.norm(np.asarray(X) - np.asarray(Xref), axis=1)
    return float(np.max(err / np.maximum(scale, 1e-300)))


def rows_for_slots(plist, slots):
    """Host copies of the list rows of the given key slots (a device gather of
    just those rows): returns (key index into `slots`, partner slot, code)."""
    s = torch.as_tensor(slots, dtype=torch.long, device=plist.offsets.device)
    off = plist.offsets[s]
    cnt = plist.counts[s].long()
    rep = torch.repeat_interleave(torch.arange(s.numel(), device=s.device), cnt)
    first = torch.cumsum(cnt, 0) - cnt
    within = torch.arange(rep.numel(), device=s.device) - first[rep]
    ent = plist.nbr[off[rep] + within].long() & 0xFFFFFFFF
    return rep.cpu().numpy(), (ent & SLOT_MASK).cpu().numpy(), (ent >> 27).cpu().numpy()


def _wrap(z, n):
    return z + n if z < 0 else (z - n if z >= n else z)


def tile_slots(start, count, nc, tc, key_cell_xyz, entries):
    """Partner slots of tiled entries (16-bit byte offsets, 16 per particle,
    into the staged neighbourhood of the key's tile), decoded on the host from the layout the
    C header states: tiles of tc cells along z; a tile's neighbourhood lists
    the runs of cells z0-1 .. z1 (periodic) of the 9 columns (cx+sx, cy+sy),
    column (sx+1)*3 + (sy+1) after column, each run in z order from z0-1.
    start, count: host int arrays of the cell grid; key_cell_xyz: packed cell
    of the key of each entry."""
    nx, ny, nz = nc
    out = np.empty(len(entries), np.int64)
    cache = {}
    for i, (c, e) in enumerate(zip(key_cell_xyz, entries)):
        cx, cy, cz = c & 1023, (c >> 10) & 1023, (c >> 20) & 1023
        z0 = (cz // tc) * tc
        key = (cx, cy, z0)
        if key not in cache:
            z1 = min(z0 + tc, nz)
            pieces = []
            for col in range(9):
                X, Y = _wrap(cx + col // 3 - 1, nx), _wrap(cy + col % 3 - 1, ny)
                slots = []
                for z in range(z0 - 1, z1 + 1):
                    cell = (X * ny + Y) * nz + _wrap(z, nz)
                    slots.extend(range(int(start[cell]), int(start[cell]) + int(count[cell])))
                pieces.extend(slots)
            cache[key] = np.asarray(pieces, np.int64)
        assert e % 16 == 0, e
        out[i] = cache[key][e // 16]
    return out


def rows_for_slots_state(e, slots):
    """rows_for_slots for an Engine's state list in either layout: returns
    (key index into `slots`, partner slot)."""
    if not int(e.state.list_tiled):
        k, p, _ = rows_for_slots(e.plist, slots)
        return k, p
    pl = e.plist
    s = torch.as_tensor(slots, dtype=torch.long, device=pl.offsets.device)
    off = pl.offsets[s]
    cnt = pl.counts[s].long()
    rep = torch.repeat_interleave(torch.arange(s.numel(), device=s.device), cnt)
    first = torch.cumsum(cnt, 0) - cnt
    within = torch.arange(rep.numel(), device=s.device) - first[rep]
    nbr16 = pl.nbr.view(torch.int16)
    ent = (nbr16[off[rep] + within].long() & 0xFFFF).cpu().numpy()
    kcell = e.grid.cell_xyz[s].cpu().numpy()[rep.cpu().numpy()]
    start = e.grid.start.cpu().numpy()
    count = e.grid.count.cpu().numpy()
    partners = tile_slots(start, count, e.grid.ncell, int(e.state.tile_cells), kcell, ent)
    return rep.cpu().numpy(), partners
