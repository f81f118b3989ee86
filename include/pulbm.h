/*
 * pulbm.h -- C ABI of libpulbm.so, the MI355X (gfx950) HIP solver for the
 * coupled phase-field + P-u lattice Boltzmann step of Otomo et al.,
 * "Lattice Boltzmann models for the hydrodynamic equations in multiphase flow
 * with high density ratio" (arXiv 2512.01027).
 *
 * The calls follow the paper's statement of the problem (Sec. II): fluid
 * properties (rho, nu of both fluids, sigma, W, M, lambda_b, body force) and
 * geometry go in, the initial phi, P, u are turned into equilibrium
 * distributions (Sec. I, the initial state is the equilibrium), the coupled
 * step is advanced N times, and phi, P, u are read back (the zeroth moment of
 * h and the P/u reconstruction of Sec. II).
 *
 * General rules
 *  - Every call returns 0 (PULBM_OK) or a negative PULBM_E* code and never
 *    throws; pulbm_last_error() then describes the failure (thread-local).
 *  - Host arrays are caller-owned, FP64, node index n = x + nx*(y + ny*z)
 *    (x fastest; 2D uses nz = 1), vector fields SoA: u[a*N + n].  They are
 *    copied; the library keeps no host pointer.
 *  - Device memory is either allocated by the library (hipMalloc) or carved
 *    from a caller-owned device arena (e.g. a torch tensor) that must outlive
 *    the case and be at least pulbm_required_bytes() long.
 *  - All work on a case is ordered on the HIP stream given at creation (NULL
 *    = the default stream).  pulbm_step() returns as soon as the launches are
 *    queued; read, diagnostics and checkpoint calls synchronise the stream.
 *  - One MI355X per process; a case lives on the device that was current at
 *    pulbm_create().
 */
#ifndef PULBM_H
#define PULBM_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PULBM_OK 0
#define PULBM_EINVAL (-1)    /* bad argument or parameter                         */
#define PULBM_ENOMEM (-2)    /* device allocation failed / arena too small        */
#define PULBM_EDEVICE (-3)   /* a HIP call failed                                 */
#define PULBM_EDIVERGED (-4) /* non-finite values found in the fields             */
#define PULBM_ESTATE (-5)    /* call out of order (e.g. step before init)         */
#define PULBM_EAGAIN (-6)    /* serving: no free slot or memory for the request   */

/* Storage precision of the distributions (compute precision in brackets). */
#define PULBM_STORE_FP64 0 /* FP64 (FP64)                                             */
#define PULBM_STORE_FP32 1 /* FP32 (FP32; pressure reconstruction and sums in FP64)   */
#define PULBM_STORE_FP16 2 /* FP16 shifted and scaled populations (FP32 compute):   */
                           /* h_j - w_j phi and g_i - w_i c_i.u / T, with phi and  */
                           /* u of the reading node at the previous step (the     */
                           /* pressure part of g is kept apart), scaled by powers */
                           /* of two                                               */
#define PULBM_STORE_BF16 3 /* BF16, the same shifted populations (FP32 compute)     */

/* Case parameters, lattice units (Sec. II; defaults of Sec. III in brackets). */
typedef struct {
    int32_t dim, nx, ny, nz;     /* dim 2 (nz = 1) or 3; every n >= 1.  Device fields pad
                                    each row to a multiple of 32 nodes; the padded count
                                    (nx rounded up to 32) * ny * nz must stay below 2^28 in
                                    FP64 storage, below 2^29 otherwise.  Host arrays are
                                    compact (x fastest, no padding).                        */
    int32_t q_hydro, q_phase;    /* 2D: 9, 9; 3D: 27 or 19, 19 (hydro D3Q27, or D3Q19 as the
                                    paper's 3D runs; phase field D3Q19)                      */
    int32_t wall[3];             /* per axis: 0 periodic, 1 no-slip walls at both ends, 2
                                    (last axis only) a wall at the low end and an open end
                                    at pressure p_top at the high end (the dam break's
                                    atmospheric top, Sec. III)                              */
    int32_t delta_theta;         /* 1: apply the delta-theta correction of Sec. II [1]      */
    int32_t store;               /* PULBM_STORE_*                                           */
    int32_t collision;           /* hydrodynamic collision: 0 the filter collision of Sec. II
                                    (Eq. LB_filter_col) [0]; 1 BGK with tau_mix (Eq.
                                    BGK_LBeq_hydroeq; less robust at high density ratio)    */
    double rho_heavy, rho_light; /* densities of the phi = 1 and phi = 0 fluids              */
    double nu_heavy, nu_light;   /* kinematic viscosities (> 0)                             */
    double sigma, W, M;          /* surface tension, interface width, mobility [M = 0.166]  */
    double lambda_bulk;          /* bulk viscosity [1/6]                                    */
    double gravity[3];           /* body force per unit mass, F_ext = rho g                 */
    int32_t block_lo[3], block_hi[3]; /* solid block (the dam break's obstacle, Sec. III):
                                    nodes lo <= x < hi on every axis; none if lo >= hi on
                                    any axis.  At least 2 nodes thick (or spanning the
                                    axis); not across a periodic boundary; not touching
                                    an open end.  Its nodes carry no fluid and read back
                                    phi = P = u = 0.                                        */
    double p_top;                /* pressure at an open end (wall = 2)                      */
} pulbm_params;

typedef struct {
    double phi_sum;     /* sum of phi over the nodes (FP64)              */
    double u_sum[3];    /* sum of u                                      */
    double rhou_sum[3]; /* sum of rho u                                  */
    double umax;        /* max |u|                                       */
    int64_t nonfinite;  /* nodes with a non-finite phi, P or u component */
    int64_t step;       /* steps taken since init                        */
} pulbm_diag;

typedef struct pulbm_case pulbm_case;

/* Device bytes a case needs (for a caller-provided arena). */
int pulbm_required_bytes(const pulbm_params* p, size_t* bytes);

/* Validate p and create a case.  dev_arena may be NULL (library allocates);
 * hip_stream may be NULL (default stream).  *out receives the handle. */
int pulbm_create(const pulbm_params* p, void* dev_arena, size_t arena_bytes, void* hip_stream,
                 pulbm_case** out);

/* Equilibrium initialisation from host phi[N], P[N], u[dim*N] (Sec. I: the
 * distributions start at equilibrium; the previous-step pressure is P). */
int pulbm_init_fields(pulbm_case* c, const double* phi, const double* P, const double* u);

/* Queue nsteps coupled steps (moments, pressure, velocity, collide+stream)
 * on the case's stream.  Returns without waiting. */
int pulbm_step(pulbm_case* c, int64_t nsteps);

/* Like pulbm_step, but waits and adds the GPU time of each of the four
 * kernels (moments, pressure, velocity, collide+stream) to ms[0..3] (HIP
 * events on the case's stream around every launch). */
int pulbm_step_timed(pulbm_case* c, int64_t nsteps, double* ms);

/* phi[N], P[N], u[dim*N] of the current state: the moment stage applied to
 * the current distributions without changing them.  Synchronises. */
int pulbm_read_fields(pulbm_case* c, double* phi, double* P, double* u);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the same phi, P, u as
 * pulbm_read_fields (bit for bit), read back without any host or device
 * allocation.  The compact FP64 fields are staged in a fixed device array of
 * the library (64 MiB on each GPU it runs on, held until the process ends),
 * so (2 + dim) * nx * ny * nz doubles must fit it: at most 1,677,721 nodes in
 * 3D, 2,097,152 in 2D (PULBM_EINVAL otherwise, before any GPU work).  Calls
 * on one GPU share that array; within a process they are serialised by a
 * lock, so calls overlapping from several threads wait for each other.
 * Synchronises the case's stream. */
int pulbm_read_fields_noalloc(pulbm_case* c, double* phi, double* P, double* u);

/* Conservation diagnostics of the current state (FP64 wave reductions).
 * Returns PULBM_EDIVERGED (with *d filled) if any value is non-finite. */
int pulbm_diagnostics(pulbm_case* c, pulbm_diag* d);

/* Restart image (distributions in their storage precision, previous-step
 * pressure, phi and u, step count, parameters).  checkpoint_bytes gives the
 * size.  pulbm_restore accepts only an image of a case with the same grid,
 * lattices, storage, walls, open end (and p_top), block and collision; its
 * section sizes must equal the case's and its step count be >= 0.  Anything
 * else is PULBM_EINVAL before a byte is copied, and the case keeps its state.
 * Fluid properties, body force and the delta-theta switch are the target
 * case's own (the image's are ignored). */
int pulbm_checkpoint_bytes(const pulbm_case* c, size_t* bytes);
int pulbm_checkpoint(pulbm_case* c, void* host_buf, size_t bytes);
int pulbm_restore(pulbm_case* c, const void* host_buf, size_t bytes);

/* Wait for all queued work of the case. */
int pulbm_sync(pulbm_case* c);
int64_t pulbm_steps_done(const pulbm_case* c);

/* Race check of the in-place AA pattern and the tile-parallel kernels:
 * order 1 makes every later launch of the case take its tiles in the
 * reverse of the usual order (the workgroup that would take the first tile
 * takes the last), so each tile runs on another workgroup, XCD and time.
 * Within a step no workgroup may read what another one writes in the same
 * launch, so results are bitwise those of order 0 (the default), which
 * restores the usual order.  Queued on the case's stream; PULBM_EINVAL for
 * a NULL case or an order other than 0 or 1. */
int pulbm_set_tile_order(pulbm_case* c, int32_t order);
void pulbm_destroy(pulbm_case* c);

/* Message of the last failed call on this thread ("" if none). */
const char* pulbm_last_error(void);

/* -------------------------------------------------------------- measurement
 * Bandwidth probe (not part of the method): copies `bytes` from device src to
 * device dst `reps` times on the HIP stream (NULL = default) with a plain
 * streaming kernel (16-byte vectors, 16 KiB per workgroup) and returns the
 * average milliseconds per copy in *ms (HIP events; one untimed copy first).
 * mode bit 0: non-temporal loads, bit 1: non-temporal stores.  bytes and
 * both pointers must be multiples of 16 and the buffers must not overlap
 * (PULBM_EINVAL otherwise).  The copy moves 2 * bytes of HBM traffic: it
 * gives the attainable read + write rate that the step's traffic is set
 * against.  Synchronises the stream. */
int pulbm_stream_copy(void* dst, const void* src, size_t bytes, int32_t mode, int32_t reps, void* hip_stream,
                      double* ms);

/* ------------------------------------------------------------------ serving
 * A batch keeps many cases resident in one device arena (the budget,
 * allocated once at creation) and advances all active cases together: each
 * launch covers the tiles of every resident case of a lattice (2D or 3D), and
 * a k-step advance is one replay of a captured HIP graph on the batch stream.
 * Each case runs exactly its requested number of steps; its arithmetic is the
 * same as a single case's, so results do not depend on which other cases
 * share the batch.  A batch uses one storage precision.
 *
 * Admissions and read-backs run on a second stream of the batch, so they
 * overlap the advances already queued.  The calls of one batch must come
 * from one thread at a time. */
typedef struct pulbm_batch pulbm_batch;

int pulbm_batch_create(size_t hbm_budget, int32_t store, int32_t max_slots, void* hip_stream,
                       pulbm_batch** out);
/* Admit a case (host FP64 initial fields) for nsteps steps.  Returns
 * PULBM_EAGAIN if no slot or not enough of the budget is free; *slot gets the
 * slot id otherwise.  p->store must equal the batch's store. */
int pulbm_batch_admit(pulbm_batch* b, const pulbm_params* p, const double* phi, const double* P,
                      const double* u, int64_t nsteps, int32_t* slot);
/* Queue ksteps steps of every active case (a captured graph per ksteps). */
int pulbm_batch_advance(pulbm_batch* b, int32_t ksteps);
/* Slots whose cases have finished; fills up to cap ids, *ndone = how many.
 * Waits for every queued advance but the newest one (for all of them when no
 * resident case has steps left), so that the newest keeps the GPU busy while
 * the caller takes and admits cases. */
int pulbm_batch_poll(pulbm_batch* b, int32_t* done_slots, int32_t cap, int32_t* ndone);
/* Read a case's phi, P, u (as pulbm_read_fields; for a case that has not
 * finished: its state after every queued advance) and free its slot.  Its
 * memory returns to the budget once the advances queued so far complete. */
int pulbm_batch_take(pulbm_batch* b, int32_t slot, double* phi, double* P, double* u);
/* Bytes of the budget in use, number of active cases. */
int pulbm_batch_usage(const pulbm_batch* b, size_t* used, int32_t* active);
void pulbm_batch_destroy(pulbm_batch* b);

#ifdef __cplusplus
}
#endif
#endif
