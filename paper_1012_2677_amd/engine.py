"""Device buffers (torch, used only for memory and streams) around the C ABI.

`Grid` and `PairList` own the arrays of md_cells / md_pairlist; `Engine` owns a
whole md_state and runs md_prepare / md_step.  Nothing here computes the
method: every step runs in the HIP library.
"""

from __future__ import annotations

import math

import numpy as np
import torch

from . import _abi as A


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else t.data_ptr()


REBUILD_RULES = {"half_skin": A.MD_REBUILD_HALF_SKIN, "dutc_ldc": A.MD_REBUILD_DUTC_LDC}


LIST_LAYOUTS = {"auto": A.MD_LIST_AUTO, "slots": A.MD_LIST_SLOTS, "half": A.MD_LIST_HALF}


BUILD_WAVES = {"auto": A.MD_BUILD_AUTO, "cell": A.MD_BUILD_CELL_WAVES, "tile": A.MD_BUILD_TILE_WAVES}


def make_params(n, box, *, eps=1.0, sigma=1.0, rc=2.5, rs=2.8, dt=0.005, precision="fp64",
                resort_every=1, rebuild_rule="half_skin", ldc_max=8192, list_layout="auto",
                tile_cells=0, step_run=0, build_waves="auto") -> A.MdParams:
    p = A.MdParams()
    p.n = int(n)
    b = np.broadcast_to(np.asarray(box, dtype=np.float64), (3,))
    for k in range(3):
        p.box[k] = float(b[k])
    p.eps, p.sigma, p.rc, p.rs, p.dt = float(eps), float(sigma), float(rc), float(rs), float(dt)
    p.precision = A.MD_MIXED if precision in ("mixed", A.MD_MIXED) else A.MD_FP64
    p.resort_every = int(resort_every)
    p.rebuild_rule = REBUILD_RULES[rebuild_rule] if isinstance(rebuild_rule, str) else int(rebuild_rule)
    p.ldc_max = int(ldc_max)
    p.list_layout = LIST_LAYOUTS[list_layout] if isinstance(list_layout, str) else int(list_layout)
    p.tile_cells = int(tile_cells)
    p.step_run = int(step_run)
    p.build_waves = BUILD_WAVES[build_waves] if isinstance(build_waves, str) else int(build_waves)
    return p


def stream_handle(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


class Workspace:
    def __init__(self, params: A.MdParams, device):
        self.nbytes = A.md_workspace_bytes(params)
        self.buf = torch.empty(max(self.nbytes, 256), dtype=torch.uint8, device=device)

    @property
    def ptr(self) -> int:
        return self.buf.data_ptr()


class Grid:
    """md_cells arrays for n particles."""

    def __init__(self, params: A.MdParams, device):
        self.ncell = A.md_cell_dims(params)
        nc = int(np.prod(self.ncell))
        n = params.n
        i32 = dict(dtype=torch.int32, device=device)
        self.cell_of = torch.empty(n, **i32)
        self.cell_xyz = torch.empty(n, **i32)
        self.count = torch.empty(nc, **i32)
        self.start = torch.empty(nc + 1, **i32)
        self.order = torch.empty(n, **i32)
        self.c = A.MdCells()
        self.fill(self.c)

    def fill(self, c: A.MdCells):
        for k in range(3):
            c.ncell[k] = self.ncell[k]
        c.cell_of = self.cell_of.data_ptr()
        c.cell_xyz = self.cell_xyz.data_ptr()
        c.count = self.count.data_ptr()
        c.start = self.start.data_ptr()
        c.order = self.order.data_ptr()


def default_cell_stride(params: A.MdParams, ncell, pooled: bool = False) -> int:
    """Entries reserved per cell: the mean (cell occupancy times the mean
    number of partners within rs) times a margin, plus 64, rounded up to 64.
    Cell blocks of their own (slot entries) must hold the fullest cell of a
    fluctuating fluid: twice the mean.  The tiled layout pools the blocks of a
    tile's cells, so its stride only has to hold the fullest tile's average:
    1.35 times the mean.  Either grows on MD_ERR_CAPACITY."""
    vol = params.box[0] * params.box[1] * params.box[2]
    rho = params.n / vol
    per_cell = params.n / float(np.prod(ncell))
    mean = per_cell * rho * (4.0 / 3.0) * math.pi * params.rs ** 3
    return int(64 * math.ceil(((1.35 if pooled else 2.0) * mean + 64.0) / 64.0))


class PairList:
    """md_pairlist arrays: ncell * cell_stride entries of 32 bits (slot
    entries), or of 16 bits when entry_bits = 16 (room for the tiled layout of
    a simulation state only)."""

    def __init__(self, params: A.MdParams, ncell, device, cell_stride: int | None = None, entry_bits: int = 32):
        n = params.n
        self.ncell = ncell
        self.device = device
        self.entry_bits = int(entry_bits)
        self.offsets = torch.empty(n, dtype=torch.int64, device=device)
        self.counts = torch.empty(n, dtype=torch.int32, device=device)
        self.status = torch.zeros(4, dtype=torch.int64, device=device)
        self.l = A.MdPairlist()
        self.resize(cell_stride or default_cell_stride(params, ncell, pooled=self.entry_bits == 16))

    def resize(self, cell_stride: int, entry_bits: int | None = None):
        self.cell_stride = int(cell_stride)
        if entry_bits is not None:
            self.entry_bits = int(entry_bits)
        entries = int(np.prod(self.ncell)) * self.cell_stride
        words = entries if self.entry_bits == 32 else (entries + 1) // 2
        self.nbr = None
        self.nbr = torch.empty(words, dtype=torch.int32, device=self.device)
        self.fill(self.l)

    def fill(self, l: A.MdPairlist):
        l.offsets = self.offsets.data_ptr()
        l.counts = self.counts.data_ptr()
        l.nbr = self.nbr.data_ptr()
        l.cell_stride = self.cell_stride
        l.capacity = self.nbr.numel()
        l.status = self.status.data_ptr()

    def grow_for(self, needed: int):
        # needed is the largest block (tiled: a tile's per-cell average) of the
        # build that overflowed, already a tail value of the fluid's
        # fluctuations: 10% above it, rounded up to 64 entries
        self.resize(int(64 * math.ceil(1.1 * needed / 64.0)))

    def handle_capacity_error(self):
        """After MD_ERR_CAPACITY from a state call: a cell block overflowed
        (status[2] set: grow the stride), or the state needs 32-bit slot
        entries in room made for 16-bit ones (widen)."""
        status = self.status.cpu()
        if int(status[2]) != 0:
            self.grow_for(int(status[1]))
        else:
            self.resize(self.cell_stride, 32)

    def rows(self):
        """Host copy of the list: (offsets, counts, entries) as numpy arrays."""
        return (self.offsets.cpu().numpy(), self.counts.cpu().numpy(), self.nbr.cpu().numpy().view(np.uint32))


class Engine:
    """One simulation state on one GPU.

    pos, vel: (N, 3) arrays (any array type numpy accepts), positions in
    [0, L)^3.  precision: "fp64" or "mixed".  resort_every: re-sort the particle
    arrays into cell order at every k-th rebuild (0 = never).  rebuild_rule:
    "half_skin" or "dutc_ldc" (DUTC, then the large-displacement check with at
    most ldc_max members).  list_layout: "auto" (in mixed precision, the tiled
    list whose force pass stages each tile's neighbourhood in LDS, whenever the
    slots are in cell order), "slots", or "half" (each pair once, Sec. 2.4:
    the partner's force added by device atomics, the integrator in a pass of
    its own; much slower on this GPU, kept for comparison); tile_cells: tile
    length along z in cells (0 = automatic); step_run: steps queued per wait
    for the device (0 = automatic, 1 = a wait after every step); build_waves:
    "auto", "cell" or "tile" (the tiled list build's waves: one per cell, or
    one per tile building its cells in turn; the same rows either way).
    """

    def __init__(self, pos, vel, box, *, eps=1.0, sigma=1.0, rc=2.5, rs=2.8, dt=0.005, precision="fp64",
                 resort_every=1, rebuild_rule="half_skin", ldc_max=8192, list_layout="auto", tile_cells=0,
                 step_run=0, build_waves="auto", device="cuda", cell_stride=None, timers=False):
        pos = np.ascontiguousarray(np.asarray(pos, dtype=np.float64))
        vel = np.ascontiguousarray(np.asarray(vel, dtype=np.float64))
        n = pos.shape[0]
        self.device = torch.device(device)
        if self.device.index is None:
            self.device = torch.device("cuda", torch.cuda.current_device())
        self.params = make_params(n, box, eps=eps, sigma=sigma, rc=rc, rs=rs, dt=dt, precision=precision,
                                  resort_every=resort_every, rebuild_rule=rebuild_rule, ldc_max=ldc_max,
                                  list_layout=list_layout, tile_cells=tile_cells, step_run=step_run,
                                  build_waves=build_waves)
        self.n = n
        self.mixed = self.params.precision == A.MD_MIXED
        dev = self.device
        f64 = dict(dtype=torch.float64, device=dev)
        self.grid = Grid(self.params, dev)
        # a re-sorted state keeps the tiled layout (16-bit entries) unless a
        # tile's neighbourhood is too crowded to stage; the list is widened
        # to slot entries only when the library asks for it
        tiled = self.params.list_layout == A.MD_LIST_AUTO and resort_every > 0
        self.plist = PairList(self.params, self.grid.ncell, dev, cell_stride, entry_bits=16 if tiled else 32)
        self.ws = Workspace(self.params, dev)
        p4 = np.zeros((n, 4))
        p4[:, :3] = pos
        self.pos = torch.from_numpy(p4).to(dev)
        self.vel = torch.from_numpy(np.ascontiguousarray(vel.T)).to(dev)
        self.id = torch.arange(n, dtype=torch.int32, device=dev)
        resort = resort_every > 0
        # second buffers: the re-sort writes all three; in FP64 every step also
        # writes its drifted positions to pos_alt (mixed: local coordinates to
        # pos32_alt) while the force pass still reads the current ones
        self.pos_alt = torch.empty_like(self.pos) if (resort or not self.mixed) else None
        self.vel_alt = torch.empty_like(self.vel) if resort else None
        self.id_alt = torch.empty_like(self.id) if resort else None
        self.force = torch.zeros((3, n), dtype=torch.float32 if self.mixed else torch.float64, device=dev)
        self.pos_ref = torch.empty((3, n), **f64)
        self.pos32 = torch.empty((n, 4), dtype=torch.float32, device=dev) if self.mixed else None
        self.pos32_alt = torch.empty_like(self.pos32) if self.mixed else None
        self.energy = torch.zeros(8, **f64)
        self.flags = torch.zeros(8, dtype=torch.int64, device=dev)
        self.host_scratch = torch.zeros(16, dtype=torch.int64, pin_memory=True)
        self.timers = A.MdTimers() if timers else None
        s = A.MdState()
        s.pos, s.vel, s.force = _ptr(self.pos), _ptr(self.vel), _ptr(self.force)
        s.pos_ref, s.pos32, s.pos32_alt, s.id = _ptr(self.pos_ref), _ptr(self.pos32), _ptr(self.pos32_alt), _ptr(self.id)
        s.pos_alt, s.vel_alt, s.id_alt = _ptr(self.pos_alt), _ptr(self.vel_alt), _ptr(self.id_alt)
        self.grid.fill(s.cells)
        self.plist.fill(s.list)
        s.energy, s.flags = _ptr(self.energy), _ptr(self.flags)
        s.host_scratch = _ptr(self.host_scratch)
        s.ws, s.ws_bytes = self.ws.ptr, self.ws.nbytes
        s.timers = C_pointer(self.timers)
        self.state = s
        self.prepared = False

    def reset(self, pos: torch.Tensor, vel: torch.Tensor):
        """Start again from device positions (N, 3) (or (N, 4)) and velocities
        (N, 3), in the original particle order, keeping every buffer: the
        arrays are copied in on the device and the next step prepares the
        state from scratch."""
        with torch.no_grad():
            self.pos[:, :3].copy_(pos[:, :3])
            self.pos[:, 3].zero_()
            self.vel.copy_(vel.t())
            self.id.copy_(torch.arange(self.n, dtype=torch.int32, device=self.device))
        s = self.state
        s.step = 0
        s.rebuilds = 0
        s.resorts = 0
        s.phase = 0
        s.list_valid = 0
        s.ldc_checks = 0
        s.ldc_kept = 0
        self.prepared = False

    # -- pointer bookkeeping after the library swapped buffers ------------------
    def _sync_pointers(self):
        s = self.state
        for cur, alt in (("pos", "pos_alt"), ("vel", "vel_alt"), ("id", "id_alt"), ("pos32", "pos32_alt")):
            t_cur, t_alt = getattr(self, cur), getattr(self, alt)
            if t_alt is not None and getattr(s, cur) == t_alt.data_ptr():
                setattr(self, cur, t_alt)
                setattr(self, alt, t_cur)

    def stream(self) -> int:
        return stream_handle(self.device)

    def prepare(self):
        with torch.cuda.device(self.device):
            for _ in range(4):
                try:
                    A.md_prepare(self.params, self.state, self.stream())
                    break
                except A.MdError as e:
                    self._sync_pointers()
                    if e.code != A.MD_ERR_CAPACITY:
                        raise
                    self.plist.handle_capacity_error()
                    self.plist.fill(self.state.list)
            self._sync_pointers()
        self.prepared = True

    def step(self, nsteps: int, sample_every: int = 0):
        """Advance nsteps; returns the energy log (k, 4) = (KE, PE, W, E) as numpy,
        one row for every step number (counted from the start) divisible by
        sample_every."""
        if not self.prepared:
            self.prepare()
        se = int(sample_every)
        log = torch.zeros((nsteps // se + 2 if se > 0 else 1, 4), dtype=torch.float64, device=self.device)
        rows = []
        done = 0
        with torch.cuda.device(self.device):
            while done < nsteps:
                before = int(self.state.step)
                err = None
                try:
                    A.md_step(self.params, self.state, nsteps - done, se, log.data_ptr(), self.stream())
                except A.MdError as e:
                    err = e
                self._sync_pointers()
                after = int(self.state.step)
                if se > 0:
                    rows.append(log[: after // se - before // se].cpu())
                done += after - before
                if err is not None:
                    if err.code != A.MD_ERR_CAPACITY:
                        raise err
                    self.plist.handle_capacity_error()
                    self.plist.fill(self.state.list)
        return torch.cat(rows).numpy() if rows else np.zeros((0, 4))

    def step_record(self, nsteps: int, sample_every: int = 0):
        """step() that also keeps the trajectory (md_step_record): returns
        (energy log, frames, built) with frames a (nsteps, N, 4) float64 device
        tensor, frame k the positions (x, y, z, 0) at which step k evaluated
        its forces, rows in the original particle order, and built a numpy
        bool array, True where step k rebuilt the pair list."""
        import ctypes

        if not self.prepared:
            self.prepare()
        se = int(sample_every)
        log = torch.zeros((nsteps // se + 2 if se > 0 else 1, 4), dtype=torch.float64, device=self.device)
        frames = torch.empty((nsteps, self.n, 4), dtype=torch.float64, device=self.device)
        built = (ctypes.c_int32 * max(nsteps, 1))()
        rows = []
        done = 0
        with torch.cuda.device(self.device):
            while done < nsteps:
                before = int(self.state.step)
                err = None
                sub = ctypes.cast(ctypes.byref(built, 4 * done), ctypes.POINTER(ctypes.c_int32))
                try:
                    A.md_step_record(self.params, self.state, nsteps - done, se, log.data_ptr(),
                                     frames[done:].data_ptr(), sub, self.stream())
                except A.MdError as e:
                    err = e
                self._sync_pointers()
                after = int(self.state.step)
                if se > 0:
                    rows.append(log[: after // se - before // se].cpu())
                done += after - before
                if err is not None:
                    if err.code != A.MD_ERR_CAPACITY:
                        raise err
                    self.plist.handle_capacity_error()
                    self.plist.fill(self.state.list)
        elog = torch.cat(rows).numpy() if rows else np.zeros((0, 4))
        return elog, frames, np.array(built[:nsteps], dtype=bool)

    def energies(self):
        """(KE, PE, W, E) at the current state (recomputes forces)."""
        out = torch.zeros(4, dtype=torch.float64, device=self.device)
        with torch.cuda.device(self.device):
            A.md_energy(self.params, self.state, out.data_ptr(), self.stream())
        return out.cpu().numpy()

    # -- views in original particle order ----------------------------------------
    def _inverse(self):
        ids = self.id.long()
        inv = torch.empty_like(ids)
        inv[ids] = torch.arange(self.n, device=self.device)
        return inv

    def positions(self) -> np.ndarray:
        return self.pos[:, :3][self._inverse()].cpu().numpy()

    def velocities(self) -> np.ndarray:
        return self.vel.T[self._inverse()].cpu().numpy()

    def forces(self) -> np.ndarray:
        return self.force.T[self._inverse()].double().cpu().numpy()

    @property
    def step_count(self) -> int:
        return int(self.state.step)

    @property
    def rebuilds(self) -> int:
        return int(self.state.rebuilds)

    @property
    def ldc_stats(self):
        """(large-displacement checks made, checks that kept the list)."""
        return int(self.state.ldc_checks), int(self.state.ldc_kept)

    def timer_dict(self):
        if self.timers is None:
            return {}
        return {name: (self.timers.ms[k], int(self.timers.launches[k])) for k, name in enumerate(A.TIMER_NAMES)}


def C_pointer(t):
    import ctypes

    return ctypes.pointer(t) if t is not None else ctypes.POINTER(A.MdTimers)()
