/*
 * md.h -- C ABI of the MI355X (gfx950) Lennard-Jones MD hot path.
 *
 * The method is that of Watanabe, Suzuki and Ito, "Efficient Implementations
 * of Molecular Dynamics Simulations for Lennard-Jones Systems": a truncated LJ
 * potential (Sec. 2.1), an inexclusive cell grid built by counting sort
 * (Sec. 2.2), a pair list with a search length rs > rc reused for several steps
 * (Sec. 2.3), a key-sorted pair list and force loop (Sec. 2.4, Sec. 3.1), a
 * cell-order re-sort of the particle arrays (Sec. 3.3) and a second-order
 * symplectic integrator in a periodic box (Sec. 4.5).
 *
 * General rules
 *   - Every pointer argument named as "device" is a device (HBM) address on the
 *     current HIP device; "host" pointers are ordinary host memory.
 *   - The caller allocates and frees every buffer, including the workspace;
 *     the library never allocates device memory (md_forces_noalloc keeps its
 *     scratch in a fixed array of the library's own, see there).
 *   - All work is enqueued on the given hipStream_t.  md_prepare, md_step,
 *     md_step_record and md_ldc_check synchronise that stream (they read
 *     device flags), md_hbm_probe waits for its timing events; every other
 *     call is asynchronous and returns only errors detectable on the host.
 *   - Return value: MD_OK (0) or a negative MD_ERR_* code; md_last_error()
 *     then returns a message (thread-local, valid until the next call).
 *   - Argument checks run on the host before any launch, so a call that fails
 *     validation enqueues nothing.
 *
 * Units: reduced LJ units, unit mass.
 *
 * Layouts (n = number of particles, slots are the current array positions):
 *   pos     device double[n][4]   (x, y, z, 0) per slot; 0 <= x < L required
 *                                 where noted (md_step maintains it)
 *   vel     device double[3][n]   x block, then y block, then z block
 *   force   device double[3][n] (MD_FP64) or float[3][n] (MD_MIXED)
 *   u, Hu   device double[3][n]   (adjoint vectors)
 */
#ifndef MD355_MD_H
#define MD355_MD_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define MD_OK             0
#define MD_ERR_ARG       (-1)  /* null pointer, n <= 0 or n >= 2^27, bad parameter   */
#define MD_ERR_BOX       (-2)  /* fewer than 3 or more than 1023 cells on an axis     */
#define MD_ERR_CAPACITY  (-3)  /* pair list does not fit: see md_pairlist.status     */
#define MD_ERR_NONFINITE (-4)  /* a force or energy became inf/NaN                    */
#define MD_ERR_HIP       (-5)  /* HIP launch/runtime failure                          */
#define MD_ERR_WORKSPACE (-6)  /* workspace smaller than md_workspace_bytes()         */

/* precision modes */
#define MD_FP64  0   /* every pair term and sum in FP64                              */
#define MD_MIXED 1   /* pair displacement, force and per-particle sums in FP32;
                        positions, velocities, integration and global sums in FP64 */

#define MD_MAX_N ((int64_t)1 << 27)   /* slots are stored in 27 bits of a list entry */

/* list layouts of the simulation state (md_params.list_layout) */
#define MD_LIST_AUTO  0   /* tiled when possible (mixed precision, slots in cell order) */
#define MD_LIST_SLOTS 1   /* always 32-bit slot entries                                 */
#define MD_LIST_HALF  2   /* 32-bit slot entries, each pair once (half stencil)          */

/* pair-list rebuild rules (md_params.rebuild_rule) */
#define MD_REBUILD_HALF_SKIN 0   /* rebuild once some particle moved more than (rs - rc)/2         */
#define MD_REBUILD_DUTC_LDC  1   /* DUTC, then the large-displacement check (Alg. alg_validity_check) */

#define MD_STEP_RUN_MAX 64       /* most steps md_step queues per host wait (md_params.step_run) */

/* waves of the tiled list build (md_params.build_waves) */
#define MD_BUILD_AUTO       0   /* a wave per tile from MD_BUILD_TILE_MIN tiles on, else a wave per cell */
#define MD_BUILD_CELL_WAVES 1   /* a wave per cell; the cells of a tile reserve their rows by atomics   */
#define MD_BUILD_TILE_WAVES 2   /* a wave per tile, building its cells one after another along z        */
#define MD_BUILD_TILE_MIN   32768

/* Model and run parameters.
 *   V(r) = 4 eps [ (sigma/r)^12 - (sigma/r)^6 + c2 (r/sigma)^2 + c0 ] for r < rc,
 *   with c2, c0 fixed by V(rc) = V'(rc) = 0 (Sec. 2.1, eq. lj_cutoff); rc and rs
 *   are absolute lengths.  Pairs with r < rs are listed (Sec. 2.3); the list is
 *   rebuilt when some particle has moved more than (rs - rc)/2 since the last
 *   build (the search-length figure of Sec. 2.3).  Cells per axis are
 *   floor(L / rs) (cell side >= rs, Sec. 2.2).
 *   resort_every: re-sort the particle arrays into cell order at every k-th
 *   rebuild (Sec. 3.3; 0 = never, 1 = every rebuild).
 *   rebuild_rule: MD_REBUILD_HALF_SKIN, or MD_REBUILD_DUTC_LDC (Sec. 2.3,
 *   Alg. alg_validity_check): a buffer rs - rc shrinks by 2 v_max dt per step
 *   (v_max the largest speed of the step's drift); while it is positive the
 *   list is valid, afterwards md_ldc_check decides each step.
 *   ldc_max: the most particles the large-displacement check takes (N_l of
 *   the algorithm); more invalidate the list outright.  0 <= ldc_max <= 2^22.
 *   list_layout: how md_prepare / md_step / md_energy store the state's list.
 *   MD_LIST_AUTO: whenever the slots are in cell order (after a re-sort), the
 *   list's cell_stride is even and every tile's neighbourhood fits (3500
 *   particles in MD_MIXED, 1950 in MD_FP64), the tiled layout: the cells
 *   are cut into tiles of tile_cells consecutive cells along z, and an entry
 *   is 16 times the index of the partner in the tile's neighbourhood (its
 *   byte offset in the copy of the runs of cells around the tile in the 9
 *   columns next to it, which the force pass stages in LDS: 16 bytes per
 *   particle in MD_MIXED, 24 in MD_FP64, where the offset is 1.5 times the
 *   entry); otherwise, and always with MD_LIST_SLOTS, entries are
 *   32-bit partner slots as in md_build_pairlist.  Both layouts hold the same
 *   pairs in the same row order.
 *   MD_LIST_HALF: every pair once (Sec. 2.4, the key/partner list with
 *   Newton's third law), in md_build_pairlist as well as in the state: the
 *   row of key i holds the partners in its own cell with a larger slot, then
 *   those in the 13 neighbour cells of stencil codes 14 .. 26, in the order
 *   of a full row (own cell, then codes 14 .. 26; slots ascending).  The force passes add each pair's force
 *   to the key in registers and to the partner with a device atomic, so the
 *   rounding of a force sum depends on the order of the atomics; in a
 *   simulation state the integrator then runs as a pass of its own.
 *   tile_cells: cells per tile along z (0 = about 200 keys per tile at the
 *   mean density in MD_MIXED, 146 in MD_FP64); clipped to [1, nz - 2].
 *   step_run: with MD_REBUILD_HALF_SKIN and a full list, the steps md_step
 *   queues before it waits for the device (0 = automatic: the steps the list
 *   is expected to last, from its age and the growth of the largest
 *   displacement, plus one, at most MD_STEP_RUN_MAX; 1 = a wait after every
 *   step).  The results do not depend on it.
 *   build_waves: how the build of a tiled list spreads its work (MD_BUILD_*).
 *   The rows are the same either way; only the order of the cells' rows
 *   inside their tile's block differs (cell order with a wave per tile, the
 *   order in which the cells finish with a wave per cell), so forces and
 *   runs do not depend on it. */
typedef struct md_params {
    int64_t n;
    double  box[3];
    double  eps, sigma;
    double  rc, rs;
    double  dt;
    int32_t precision;     /* MD_FP64 or MD_MIXED */
    int32_t resort_every;
    int32_t rebuild_rule;  /* MD_REBUILD_HALF_SKIN or MD_REBUILD_DUTC_LDC */
    int32_t ldc_max;
    int32_t list_layout;   /* MD_LIST_AUTO, MD_LIST_SLOTS or MD_LIST_HALF */
    int32_t tile_cells;    /* 0 = automatic, else 1 .. 1023 */
    int32_t step_run;      /* 0 = automatic, else 1 .. MD_STEP_RUN_MAX steps per wait */
    int32_t build_waves;   /* MD_BUILD_AUTO, MD_BUILD_CELL_WAVES or MD_BUILD_TILE_WAVES */
} md_params;

/* Cell grid (Sec. 2.2): GridParticleNumber = count, GridPointer = start,
 * GridList = order.  Cell id of a slot: (cx * ny + cy) * nz + cz with
 * cx = min(floor(x * nx / L), nx - 1).
 *   cell_of   device int32[n]      cell id of each slot
 *   cell_xyz  device int32[n]      packed cell coords cx | cy << 10 | cz << 20
 *   count     device int32[nc]     particles per cell
 *   start     device int32[nc+1]   exclusive prefix sum of count; start[nc] = n
 *   order     device int32[n]      slots sorted by cell, stable (ascending slot
 *                                  within a cell)
 *   sorted    host flag: 1 when the slots themselves are in cell order (after a
 *             re-sort), so that cell c holds slots start[c] .. start[c+1]-1; the
 *             library sets it, md_bin_cells clears it.                       */
typedef struct md_cells {
    int32_t  ncell[3];
    int32_t  sorted;
    int32_t* cell_of;
    int32_t* cell_xyz;
    int32_t* count;
    int32_t* start;
    int32_t* order;
} md_cells;

/* Key-sorted pair list (Sec. 2.4: KeyPointer / SortedList), full (both
 * directions): the row of key slot i is nbr[offsets[i] .. offsets[i]+counts[i]).
 * Each entry is (partner slot) | (stencil code << 27), where the stencil code
 * (sx+1)*9 + (sy+1)*3 + (sz+1) names the neighbour cell of the partner relative
 * to the key's cell at build time (s in {-1,0,1}^3).  Rows list the partners
 * cell by cell, the key's own cell (code 13) first, then codes 14 .. 26 and
 * 0 .. 12, each cell's partners in ascending slot.  Rows of the keys of cell c live in
 * the block nbr[c*cell_stride .. (c+1)*cell_stride).
 *   offsets   device int64[n]
 *   counts    device int32[n]
 *   nbr       device uint32[capacity], 1 <= cell_stride <= 2^29;
 *             capacity >= nc * cell_stride for slot entries (every call
 *             but md_prepare / md_step / md_energy), and for a simulation
 *             state whose list is tiled (16-bit entries, see md_state)
 *             capacity >= nc * cell_stride / 2 (rounded up) is enough; should
 *             such a state need slot entries, md_prepare / md_step return
 *             MD_ERR_CAPACITY with status[2] clear (grow nbr and call again)
 *   status    device int64[4]: [0] total entries, [1] largest per-cell block,
 *             [2] 1 if some cell block overflowed cell_stride (list invalid),
 *             [3] reserved.
 *   tiled     set by the library: 0 after md_build_pairlist (the entries
 *             above); 1 when md_prepare / md_step left the tiled layout of a
 *             simulation state in this list (see md_state).  md_forces,
 *             md_hvp, md_param_grad and md_adjoint_kick read slot entries
 *             only and return MD_ERR_ARG for a tiled list.
 *   half      set by the library: 1 when the rows hold each pair once
 *             (md_params.list_layout = MD_LIST_HALF: a key's row keeps the
 *             partners of stencil code 13 with a larger slot and those of
 *             codes 14 .. 26).  md_forces takes half lists; md_hvp,
 *             md_param_grad and md_adjoint_kick return MD_ERR_ARG for them. */
typedef struct md_pairlist {
    int64_t*  offsets;
    int32_t*  counts;
    uint32_t* nbr;
    int64_t   cell_stride;
    int64_t   capacity;
    int64_t*  status;
    int32_t   tiled;
    int32_t   half;
} md_pairlist;

/* Per-kernel-class timers filled by md_step when md_state.timers != NULL:
 * HIP-event time summed over launches, in milliseconds. */
enum { MD_T_FORCE = 0, MD_T_INTEGRATE, MD_T_BIN, MD_T_RESORT, MD_T_BUILD, MD_T_REDUCE, MD_T_CHECK, MD_T_COUNT };
typedef struct md_timers {
    double  ms[MD_T_COUNT];
    int64_t launches[MD_T_COUNT];
} md_timers;

/* Whole simulation state for md_prepare / md_step / md_energy.
 *   pos, vel, id: current arrays; pos_alt, vel_alt, id_alt: second buffers,
 *   swapped with the current ones by the library (read the pointers back
 *   after a call).  The re-sort writes all three; in MD_FP64 md_step also
 *   writes each step's drifted positions to pos_alt (the force pass still
 *   reads the old ones), so pos_alt is required in MD_FP64 and vel_alt /
 *   id_alt only when resort_every > 0.  pos_ref: device double[3][n],
 *   positions at the last build.  pos32, pos32_alt: device float[n][4],
 *   MD_MIXED only (NULL in MD_FP64): coordinates relative to each slot's cell
 *   corner at the last build, with the packed cell coordinates
 *   (cx | cy << 10 | cz << 20) as the bits of the fourth float, and the
 *   second buffer md_step writes the drifted coordinates to (swapped like
 *   pos / pos_alt).
 *   force: after md_prepare, md_energy and at the end of md_step, the forces
 *   at the current positions; inside a run they are consumed by the fused
 *   kicks and not stored.
 *   energy: device double[8]: KE, PE, W, E at the last sampled step, then
 *   the largest squared displacement since the last build and the largest
 *   squared drift speed of the last step, reserved.
 *   flags: device int64[8]: [0] non-finite force seen, others reserved.
 *   host_scratch: host int64[16] (pinned recommended) for flag read-back.
 *   ws: device workspace of ws_bytes >= md_workspace_bytes().
 *   step, rebuilds, resorts: host counters; phase: 0 = (q, v, F) at a whole
 *   step, 1 = stopped after a drift (resumed by the next md_step), 2 = arrays
 *   re-sorted by md_resort (md_prepare needed).
 *   dutc_buffer: remaining DUTC buffer length (MD_REBUILD_DUTC_LDC; reset to
 *   rs - rc at each build); ldc_checks, ldc_kept: large-displacement checks
 *   made, and those that kept the list.
 *   list_tiled: 1 when st->list holds the tiled layout (set by the library):
 *   nbr is then read as uint16 entries, offsets count uint16 units, and the
 *   cells of a tile share one pooled block: ((uint16_t*)nbr)[c0*cell_stride
 *   .. (c0 + k)*cell_stride) for a tile of k cells whose first cell is c0.
 *   Each cell's rows lie together in the pool (a cell takes its slice when
 *   its rows are made, so the order of the slices varies from build to
 *   build; the rows themselves do not).  status[1] then gives the stride the
 *   fullest tile needs (its entries over its cells, rounded up) and status[2]
 *   is set when some tile's pool overflowed.  Each row starts at an even
 *   entry (a row of odd length is followed by one entry naming the stand-in
 *   just past the tile's neighbourhood, counted in the list status but not
 *   in the row's count); tile_stage:
 *   the largest neighbourhood of a tile, in particles; tile_cells: the tile
 *   length along z in cells. */
typedef struct md_state {
    double*   pos;
    double*   vel;
    void*     force;
    double*   pos_ref;
    float*    pos32;
    float*    pos32_alt;
    int32_t*  id;
    double*   pos_alt;
    double*   vel_alt;
    int32_t*  id_alt;
    md_cells    cells;
    md_pairlist list;
    double*   energy;
    int64_t*  flags;
    int64_t*  host_scratch;
    void*     ws;
    size_t    ws_bytes;
    md_timers* timers;
    int64_t   step;
    int64_t   rebuilds;
    int64_t   resorts;
    int32_t   phase;
    int32_t   list_valid;
    double    dutc_buffer;
    int64_t   ldc_checks;
    int64_t   ldc_kept;
    int32_t   list_tiled;
    int32_t   tile_stage;
    int32_t   tile_cells;
    int32_t   reserved;
} md_state;

/* Host-only: cells per axis for these parameters.  MD_ERR_BOX when an axis
 * has fewer than 3 or more than 1023 cells. */
int md_cell_dims(const md_params* p, int32_t ncell[3]);

/* Host-only: device workspace bytes needed by every call below for p. */
size_t md_workspace_bytes(const md_params* p);

/* Periodic packing of user coordinates: pos[i] = (wrap(q[i][0]), wrap(q[i][1]),
 * wrap(q[i][2]), 0) with wrap(x) = x - L floor(x / L) folded into [0, L)
 * (periodic boundaries on all axes, Sec. 4.5).  q: device double[n][3];
 * pos: device double[n][4] (may not alias q). */
int md_pack_positions(const md_params* p, const double* q, double* pos, hipStream_t stream);

/* Cell grid of pos (Sec. 2.2): label each slot with its cell, count per cell,
 * prefix-sum the counts, place slots by cell in ascending slot order.
 * pos: device double[n][4] with 0 <= x < L.  Fills cells (which must point to
 * arrays of the sizes in md_cells) and clears cells->sorted.  Results are
 * deterministic and equal to a sequential stable counting sort. */
int md_bin_cells(const md_params* p, const double* pos, md_cells* cells,
                 void* ws, size_t ws_bytes, hipStream_t stream);

/* Re-sort (Sec. 3.3): permute st->pos, vel, id into cell order using
 * st->cells (from md_bin_cells on st->pos), writing the *_alt arrays and then
 * swapping the pointers; rewrites cells->cell_of / cell_xyz in the new slot
 * order, sets cells->sorted, copies the positions into pos_ref and, in mixed
 * mode, fills pos32.  cells->order keeps the old slot of each new slot.
 * The pair list and the forces then refer to the old order: md_step refuses
 * to run until md_prepare has been called again (md_step re-sorts by itself
 * at rebuilds when resort_every > 0). */
int md_resort(const md_params* p, md_state* st, hipStream_t stream);

/* Pair list (Sec. 2.3-2.4): for every slot i, all partners j != i whose
 * minimum-image distance satisfies r^2 < rs^2, with
 *   d = q_j - q_i per axis, d -= L * rint(d / L),
 *   r^2 = fma(dz, dz, fma(dy, dy, dx * dx))   (FP64, bit-exact),
 * found among the 27 cells around the key's cell.  cells must come from
 * md_bin_cells (and md_resort, if applied) on the same pos.  Overflow of a cell
 * block is reported in list->status ([2] = 1, [1] = the stride needed).
 * With p->list_layout = MD_LIST_HALF the rows hold each pair once (the own
 * cell's partners with a larger slot, then stencil codes 14 .. 26, found among
 * those 14 cells) and list->half is set to 1; otherwise to 0. */
int md_build_pairlist(const md_params* p, const double* pos, const md_cells* cells,
                      md_pairlist* list, void* ws, size_t ws_bytes, hipStream_t stream);

/* Forces (Sec. 3.1-3.2): for every listed pair with r < rc (strict;
 * branch-free select), F_i -= g d with d = q_j - q_i and g = -V'(r)/r.
 * force: device double[3][n] (MD_FP64) or float[3][n] (MD_MIXED).
 * pe_w: device double[2] receiving PE = sum_pairs V and the virial
 * W = sum_pairs g r^2, or NULL to skip the energy terms.  pos may have moved
 * since the list was built as long as no particle moved more than (rs-rc)/2.
 * A half list (list->half) adds each pair to both ends, the partner's share
 * F_j += g d by a device atomic into force (cleared first on the stream), so
 * the rounding of each force sum depends on the order of the atomics. */
int md_forces(const md_params* p, const double* pos, const md_cells* cells,
              const md_pairlist* list, void* force, double* pe_w,
              void* ws, size_t ws_bytes, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): md_forces
 * with its workspace taken from a fixed scratch array inside the library
 * instead of a ws argument, for at most MD_NOALLOC_MAX_N particles (larger n:
 * MD_ERR_ARG, nothing launched).  The array holds 16 bytes per particle of
 * local coordinates (mixed precision), the per-block energy partials and a
 * flag word: 16 MiB + 64 KiB + 256 B on each device the library runs on,
 * kept until the process ends.  The call allocates and frees nothing; the
 * caller passes every input and output as for md_forces, whose results it
 * gives bit for bit.  Every call on one device shares that device's array
 * (the call clears what must start at zero), so calls on one device that
 * overlap in time, on different streams or from different threads, race:
 * order them on one stream. */
#define MD_NOALLOC_MAX_N ((int64_t)1 << 20)
int md_forces_noalloc(const md_params* p, const double* pos, const md_cells* cells,
                      const md_pairlist* list, void* force, double* pe_w, hipStream_t stream);

/* Large-displacement check (Sec. 2.3, Alg. alg_validity_check) of a list
 * built at pos_ref, at positions pos: the particles whose displacement
 * |minimg(q - q_ref)| exceeds t = (rs - rc) - max displacement - 1e-12 are
 * members (all of them when t < 0; the test is made on squares,
 * d2 > t^2, with d2 = fma(dz,dz, fma(dy,dy, dx*dx))); more than p->ldc_max
 * members invalidate the list, otherwise it is invalid iff some pair of
 * members has old squared distance >= rs^2 and new squared distance < rc^2.
 * pos: device double[n][4]; pos_ref: device double[3][n].  Results go to host
 * memory: *valid (1 or 0), *members, *dmax2 (largest squared displacement).
 * Synchronises the stream. */
int md_ldc_check(const md_params* p, const double* pos, const double* pos_ref, int32_t* valid,
                 int64_t* members, double* dmax2, void* ws, size_t ws_bytes, hipStream_t stream);

/* Bin, (re-sort if resort_every > 0), build the list and evaluate forces and
 * energies at the current positions; leaves st at phase 0.  Synchronises.
 * MD_ERR_CAPACITY: st->list.status holds the stride needed. */
int md_prepare(const md_params* p, md_state* st, hipStream_t stream);

/* nsteps of velocity Verlet (kick-drift-kick, unit mass; Sec. 4.5):
 *   v += (dt/2) F;  q = wrap(q + dt v);  [rebuild if max displacement since
 *   the last build exceeds (rs - rc)/2];  F = F(q);  v += (dt/2) F.
 * Inside a run the second half kick, the next step's first half kick and its
 * drift run in the force pass (two separate roundings for the two kicks).
 * Every sample_every steps (counted from st->step) the row
 * energy_log[k][0..3] = (KE, PE, W, KE + PE) is written (device double
 * array; NULL to skip; sample_every <= 0 samples nothing).
 * With MD_REBUILD_HALF_SKIN and a full list the rebuild decision is taken on
 * the device: steps are queued in runs (md_params.step_run), a small pass
 * after each step sets a device flag once the next step must rebuild, the
 * passes of the run's later steps then do nothing, and the host waits once
 * per run and once per rebuild, resuming where the run stopped.  With
 * MD_REBUILD_DUTC_LDC or a half list it waits once per step.
 * On MD_ERR_CAPACITY the state stops in phase 1 with st->step steps done;
 * grow the list and call md_step again.
 * MD_ERR_NONFINITE stops after the step that produced a non-finite force. */
int md_step(const md_params* p, md_state* st, int64_t nsteps, int64_t sample_every,
            double* energy_log, hipStream_t stream);

/* md_step that also keeps the trajectory, for the checkpointed reverse sweep
 * of trajectory gradients (which recomputes a segment of steps from its
 * checkpoint and needs every state of it and the states its pair lists were
 * built at).  For step k of the call (k = 0 .. nsteps-1):
 *   traj + 4*n*k: device double[n][4], the positions at which step k
 *     evaluates its forces (after its drift), in the particles' original
 *     order (row id holds particle id), as (x, y, z, 0): the layout of pos,
 *     so a frame can be given to md_bin_cells / md_hvp / md_adjoint_kick as
 *     it is;
 *   built[k]: host int32, 1 when step k rebuilt the pair list (at those
 *     positions), else 0.
 * Rows k at or past the step where the call stops with an error are not
 * written.  Otherwise as md_step. */
int md_step_record(const md_params* p, md_state* st, int64_t nsteps, int64_t sample_every,
                   double* energy_log, double* traj, int32_t* built, hipStream_t stream);

/* Kinetic, potential, virial and total energy at the current state:
 * out: device double[4] = (KE, PE, W, KE + PE).  Recomputes the forces. */
int md_energy(const md_params* p, md_state* st, double* out, hipStream_t stream);

/* Hessian-vector product of U = sum_pairs V (adjoint of the force field):
 * Hu_i = sum_j d^2U/dq_i dq_j u_j, over listed pairs with r < rc, FP64.
 * dparam: device double[2] = u . dF/d(eps, sigma) (F = -grad U), or NULL.
 * u, Hu: device double[3][n]. */
int md_hvp(const md_params* p, const double* pos, const md_cells* cells,
           const md_pairlist* list, const double* u, double* Hu, double* dparam,
           void* ws, size_t ws_bytes, hipStream_t stream);

/* One fused adjoint pass (FP64) for reverse-mode sweeps of the integrator:
 *   out_i  = alpha out_i + beta (H u)_i + gamma F_i          (F = -grad U)
 *   acc[k] += cu u . dF/dtheta_k + cU dU/dtheta_k            (theta = eps, sigma)
 *   u_out_i = u_i + dt out_i   (the updated out; skipped when u_out is NULL)
 * coef = {alpha, beta, gamma, cu, cU}; dt is p->dt.  The reverse of one
 * velocity-Verlet step is two calls: the second kick at q' with
 * (1, -h, -w, h, w) and u_out (the drift of the velocity adjoint), then the
 * first kick at q with (1, -h, 0, h, 0), h = dt/2 and w the observable
 * weight.  u, out, u_out: device double[3][n] (distinct); acc: device
 * double[2], accumulated in a fixed order. */
int md_adjoint_kick(const md_params* p, const double* pos, const md_cells* cells,
                    const md_pairlist* list, const double* u, double* out, double* u_out,
                    const double coef[5], double* acc, void* ws, size_t ws_bytes,
                    hipStream_t stream);

/* dU/deps and dU/dsigma of the potential energy (FP64), into device double[2]. */
int md_param_grad(const md_params* p, const double* pos, const md_cells* cells,
                  const md_pairlist* list, double* dU, void* ws, size_t ws_bytes,
                  hipStream_t stream);

/* Message for the last non-OK status on this thread. */
const char* md_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MD355_MD_H */
