/*
 * dem.h -- C ABI of libdem.so: one timestep of soft-sphere DEM on an AMD
 * Instinct MI355X (gfx950), after Washizawa & Nakahara, "Parallel Computing
 * of Discrete Element Method on GPU" (arXiv:1301.1714).
 *
 * The problem (Sec. 3 and Sec. 4.2): particles with position x, velocity v,
 * angular velocity w, radius r and mass m; a contact law with spring,
 * damping and friction parameters (Eqs. 2-10, or the simple law of Eq. 1);
 * walls treated as particles of infinite radius (Step 8); a time step dt.
 * One step runs Steps 1-8 of Sec. 4.2: update (kick-drift), cell hash,
 * sort by cell, reorder, 27-cell sweep (Eq. 12), pair and wall forces, and
 * the closing half kick.
 *
 * Conventions shared by every call:
 *  - Host arrays are borrowed for the duration of the call; per-particle
 *    vectors are row-major n x 3 (x0 y0 z0 x1 ...), FP64, in the caller's
 *    particle order ("original order"; particle k has id k).
 *  - Device memory: the caller allocates one workspace of at least
 *    dem_workspace_bytes() bytes (any device allocation, 256-byte aligned)
 *    and keeps it alive until dem_destroy().  The library never allocates
 *    device memory itself.
 *  - Streams: every device operation is enqueued on the hipStream_t given to
 *    dem_create() (NULL = the legacy default stream).  dem_step() is
 *    asynchronous; every call that returns host data synchronises that stream.
 *  - Errors: status codes only, nothing throws across the ABI.  Errors found
 *    on the device (contact-table overflow, particle out of domain,
 *    non-finite force) are sticky: they are reported by the next synchronous
 *    call and by every call after it.
 *  - Radii are rounded to FP32 on input.
 *  - Thread safety: calls on one system must not overlap; distinct systems
 *    are independent.
 */
#ifndef DEM_H
#define DEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DEM_OK = 0,
    DEM_E_INVALID = -1,          /* bad argument or parameter */
    DEM_E_WORKSPACE = -2,        /* workspace missing or too small */
    DEM_E_CONTACT_OVERFLOW = -3, /* more contacts than the contact list can hold (see dem_params) */
    DEM_E_OUT_OF_DOMAIN = -4,    /* a particle went more than one cell outside the box */
    DEM_E_NONFINITE = -5,        /* non-finite state or force */
    DEM_E_HIP = -6,              /* a HIP runtime call failed */
    DEM_E_STATE = -7,            /* system handle unusable (destroyed or failed) */
    DEM_E_CAPACITY = -9          /* caller's output array too small; *n_out holds the size needed */
} dem_status;

typedef enum {
    DEM_LAW_LINEAR = 0, /* Eqs. 2-7, 10 with constant kn, kt */
    DEM_LAW_HERTZ = 1,  /* Eqs. 2-10: kn, kt are C_kn, C_kt of Eqs. 8-9 */
    DEM_LAW_SIMPLE = 2  /* Eq. 1: F = -k_sp d n - k_da v - k_sh v_t with v_t = v - (v.n) n (the
                           tangential part of v, Sec. 3), no torque, no history */
} dem_law;

/* Optional contact terms (dem_params.terms), each added to the practical
 * law's result on its own; the paper asks that a force term can be added or
 * removed without touching the rest of the code (Sec. 4), and names none of
 * these.  Not with DEM_LAW_SIMPLE. */
typedef enum {
    DEM_TERM_COHESION = 1, /* a constant pull `cohesion` (N) along n, towards the partner or the wall,
                              while the bodies overlap (outside Eq. 5's limit) */
    DEM_TERM_ROLLING = 2   /* rolling resistance: a couple -rolling_mu R |F_n| w_rel / |w_rel| on the
                              owner and its opposite on the partner, w_rel = w_i - w_j (w_j = 0 for a
                              wall), R of Eqs. 8-9 (r_i for a wall), |F_n| of Eq. 4 */
} dem_term;

typedef enum {
    DEM_PREC_FP64 = 0,  /* everything FP64 (radii FP32) */
    DEM_PREC_MIXED = 1  /* FP64 positions and reductions; FP32 v, w, forces, history */
} dem_precision;

/* A finite wall (for Sec. 5's box with a slit at its bottom: two plates side
 * by side): the rectangle of the plane x[axis] = at spanning lo[0]..hi[0]
 * along axis (axis + 1) % 3 and lo[1]..hi[1] along axis (axis + 2) % 3, of no
 * thickness.  Like the walls of Step 8 it is a body of infinite radius and
 * mass at rest: a sphere touches it where the rectangle's nearest point is
 * closer than its radius (d^2 < r^2, FP64, no FMA); n points from the centre
 * to that point, the overlap is r - d, R = r and M = m.  Plate k is wall
 * 6 + k (contact key -7 - k). */
#define DEM_MAX_PLATES 4
typedef struct {
    int32_t axis;     /* 0, 1 or 2 */
    int32_t reserved; /* 0 */
    double at;
    double lo[2], hi[2];
} dem_plate;

/* Parameters of one system.  Sec. 3 names the contact-law inputs; the rest
 * (box, walls, gravity, cell, capacity, precision) is the setting of Sec. 4. */
typedef struct {
    double box_lo[3], box_hi[3]; /* domain; the grid covers exactly this box */
    uint32_t wall_mask;          /* bit 2a: wall at box_lo[a]; bit 2a+1: wall at box_hi[a] */
    int32_t law;                 /* dem_law */
    double gravity[3];           /* m/s^2, added once per particle */
    double dt;                   /* time step, > 0 */
    double density;              /* m = density 4/3 pi r^3, I = 2/5 m r^2 */
    double kn, kt;               /* normal / tangential spring (Hertz: C_kn, C_kt) */
    double restitution;          /* e in (0, 1]; alpha = -2 ln e / sqrt(pi^2 + ln^2 e) (Eq. 10) */
    double eta_t_ratio;          /* tangential damping = eta_t_ratio * normal damping (Eq. 4) */
    double mu;                   /* Coulomb coefficient (Eq. 5), >= 0 */
    double simple_k[3];          /* k_sp, k_da, k_sh of Eq. 1 (DEM_LAW_SIMPLE only) */
    double cell_size;            /* requested cell width (Sec. 4.1), >= 2 max radius */
    int32_t contacts_per_particle; /* capacity of the contact lists, 1..64: the most contacts one
                                      particle may own -- partners after it in the sorted order
                                      (each pair is owned by its lower slot) plus its walls.  In
                                      the sorted order a particle may also touch at most 32
                                      partners before it.  Device memory grows with it (about
                                      this many x 84 bytes per particle in mixed precision) */
    int32_t precision;           /* dem_precision */
    int32_t tile_cells;          /* detection launch shape: 0 = one lane per particle reading
                                    neighbours through the caches; -1 = one wave64 per run
                                    of 8 cells along x, the candidates of a cell in the
                                    lanes and its particles in turn, prefilter survivors
                                    compacted by ballot and decided 64 at a time; 1..32 =
                                    workgroups over runs of this many cells along x,
                                    neighbours staged in LDS.  Changes only speed, never
                                    the contacts found */
    int32_t cell_divisor;        /* k in 1..2: the grid's cells are cell_size / k wide and a
                                    particle sweeps the (2k + 1)^3 cells around its own
                                    (k = 1: the 27 cells of Eq. 12).  Finer cells cover the
                                    same contact distance with fewer candidates.  The
                                    contacts found never change; the sorted order, and so
                                    the rounding of the sums, does.  k > 1 needs
                                    tile_cells = 0 */
    int32_t max_materials;       /* 0..16: the most materials dem_set_materials may give the
                                    system (0: one material, the constants above; device
                                    memory grows by 8 bytes per particle when > 0) */
    uint32_t terms;              /* dem_term bits (0: the paper's law alone) */
    double cohesion;             /* DEM_TERM_COHESION: the pull (N), finite */
    double rolling_mu;           /* DEM_TERM_ROLLING: the coefficient, >= 0 */
    int32_t nplates;             /* finite walls in plates[], 0..DEM_MAX_PLATES */
    int32_t reserved;            /* 0 */
    dem_plate plates[DEM_MAX_PLATES];
} dem_params;

typedef struct dem_system dem_system; /* opaque host-side handle */

/* Device bytes needed for n particles with these parameters (grid size,
 * capacity and precision all enter): the state of Sec. 4.1's data structure
 * (particle properties, the correspondence maps CM / SCM / SCCM of Eq. 11,
 * the cell starts) in the sorted order of Step 4, the contact lists of Steps
 * 5-8, the tangential history of Eq. 7 (two generations) and the per-step
 * force records.  Errors: DEM_E_INVALID. */
dem_status dem_workspace_bytes(const dem_params *p, int64_t n, size_t *bytes);

/* Create a system from host arrays (original order).
 *   x, v, omega : n x 3; r : n (rounded to FP32).
 *   F0, T0      : n x 3 contact force / torque of the state (from
 *                 dem_read_state, for an exact restart) or both NULL: then
 *                 they are evaluated on the state with the given history,
 *                 and that evaluation's new history is not kept.
 *   hist_pairs  : n_hist x 2 keys (a, b), a < b, of the tangential history
 *                 of pair contacts, or (a, -1-w) for wall w; hist_dt its
 *                 n_hist x 3 tangential displacements seen from a (Eq. 7).
 *                 n_hist = 0 and NULLs for none.
 *   workspace   : device memory of ws_bytes >= dem_workspace_bytes().
 *   hip_stream  : hipStream_t for all work of this system.
 * Synchronous.  Errors: DEM_E_INVALID (parameters, radii, keys, cell narrower
 * than the largest contact distance), DEM_E_WORKSPACE, DEM_E_NONFINITE,
 * DEM_E_OUT_OF_DOMAIN, DEM_E_CONTACT_OVERFLOW, DEM_E_HIP.  n <= 2^31 / 64. */
dem_status dem_create(const dem_params *p, int64_t n, const double *x, const double *v, const double *omega,
                      const double *r, const double *F0, const double *T0, int64_t n_hist,
                      const int64_t *hist_pairs, const double *hist_dt, void *workspace, size_t ws_bytes,
                      void *hip_stream, dem_system **out);

/* dem_create with no workspace argument, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation.  The workspace is a fixed array of
 * dem_static_workspace_capacity() bytes (64 MiB) in the library's device
 * code, one per device, which that device holds from the loading of the
 * library's code object until the process ends; this call allocates no
 * device memory (no hipMalloc, hipFree or other allocating call).
 *   The device is the one current at the call, and hip_stream must belong
 *   to it.
 *   One such system per device at a time: both would use the one array, so
 *   while a system made by this call lives (until dem_destroy, which waits
 *   for its stream) another call on the same device returns DEM_E_STATE.
 *   Calls on the system itself must not overlap, as for any system.
 *   Nothing is inherited from the array's earlier contents: everything that
 *   must start at zero is cleared by this call.
 * Arguments other than the workspace, results and errors as dem_create,
 * plus DEM_E_WORKSPACE when dem_workspace_bytes(p, n) exceeds the
 * capacity. */
dem_status dem_create_static(const dem_params *p, int64_t n, const double *x, const double *v,
                             const double *omega, const double *r, const double *F0, const double *T0,
                             int64_t n_hist, const int64_t *hist_pairs, const double *hist_dt, void *hip_stream,
                             dem_system **out);

/* Bytes of the per-device array behind dem_create_static. */
size_t dem_static_workspace_capacity(void);

/* Enqueue nsteps kick-drift-kick steps (Sec. 4.2, Steps 1-8 each).
 * Asynchronous; returns the sticky error if one is already known. */
dem_status dem_step(dem_system *s, int64_t nsteps);

/* Contact force and torque (gravity excluded) on every particle of the
 * current state with the committed history, in original order: Steps 2-8 of
 * Sec. 4.2 without the update of Step 1 (Eqs. 2-10 or Eq. 1 for pairs, Step
 * 8 for walls, the torque of Eq. 3); nothing is committed.  F, T: n x 3.
 * Synchronous. */
dem_status dem_forces(dem_system *s, double *F, double *T);

/* Current state in original order: the particle properties of Sec. 4.1
 * (x, v, omega) as Step 1 last updated them.  Any pointer may be NULL.  F, T
 * are the contact forces of the last evaluation (those the next step's first
 * half kick uses).  Synchronous. */
dem_status dem_read_state(dem_system *s, double *x, double *v, double *omega, double *F, double *T);

/* Committed tangential history: n_out entries, keys (a, b) as in dem_create,
 * sorted by (a, b) ascending as signed integers, with their n x 3 delta_t.
 * If cap < *n_out nothing is written and DEM_E_CAPACITY is returned.
 * Synchronous. */
dem_status dem_read_contacts(dem_system *s, int64_t cap, int64_t *n_out, int64_t *pairs, double *delta_t);

/* Contacts of the current positions (Steps 5-8 detection: pairs a < b with
 * d^2 < (r_a + r_b)^2, walls as (a, -1-w)), sorted like dem_read_contacts.
 * Synchronous. */
dem_status dem_contacts(dem_system *s, int64_t cap, int64_t *n_out, int64_t *pairs);

/* Collision-detection grid of the current positions (Sec. 4.1, Eq. 11):
 * cell_of_id[k] = CM[k]; id_at_slot[j] = SCCM[j] (ids sorted by (cell, id));
 * cell_start: ncell + 1 entries, cell c holds slots [start[c], start[c+1]).
 * Any pointer may be NULL.  Synchronous. */
dem_status dem_read_grid(dem_system *s, int32_t *cell_of_id, int32_t *id_at_slot, int32_t *cell_start);

/* Cells per axis (x fastest in the cell index); ncell = product. */
dem_status dem_grid_dims(dem_system *s, int32_t dims[3]);

/* FP64 diagnostics of the current state (totals the method conserves or
 * dissipates: the momentum of Step 1's update, the kinetic energies of
 * translation and of the rotation driven by Eq. 3, the potential energy of
 * gravity and the elastic energy stored by the springs of Eq. 4, Hertz's
 * 2/5 K delta^(5/2) for Eqs. 8-9), reduced in a fixed order:
 *  out[0..2] momentum sum m v   out[3] kinetic energy   out[4] rotational
 *  kinetic energy   out[5] potential energy -sum m g.(x - box_lo)
 *  out[6] elastic energy of the current contacts (normal spring energy plus
 *  1/2 k_t |delta_t|^2 with the committed history)   out[7] pair contacts
 *  out[8] wall contacts   out[9] largest overlap.  Synchronous. */
dem_status dem_diagnostics(dem_system *s, double out[10]);

/* Replace the radii (original order, rounded to FP32), e.g. to grow a packing
 * by steps.  Takes effect at the next step; the stored forces are not
 * re-evaluated.  Errors: DEM_E_INVALID (a radius <= 0 or not finite, or twice
 * the largest radius wider than cell_size).  Synchronous. */
dem_status dem_set_radii(dem_system *s, const double *r);

/* Material-pair table (Sec. 3: the constants C_kn, C_kt and alpha of
 * Eqs. 8-10 carry the indices i, j of the two bodies in contact; here the
 * Coulomb coefficient of Eq. 5 does too).
 *   ntypes     : materials, 1 <= ntypes <= p->max_materials; 0 goes back to
 *                the parameters' one material.
 *   table      : ntypes x ntypes rows of 4 doubles (kn, kt, restitution,
 *                mu) -- the parameters of the same names for a particle of
 *                material t touching one of material u at row t * ntypes + u;
 *                it must be symmetric (the pair's constants do not depend on
 *                the side looked from).  Linear law: the springs; Hertz: C_kn,
 *                C_kt; restitution in (0, 1] sets alpha as in dem_params.  The
 *                simple law (Eq. 1) keeps its own constants.
 *   type       : n materials in original order, 0 <= type[i] < ntypes.
 *   wall_type  : material of every wall, 0 <= wall_type < ntypes.
 * The contact and wall forces of the current state are then evaluated again
 * with the committed history (which is kept), so that the stored forces are
 * those of a system created with these materials.  Synchronous.  Errors:
 * DEM_E_INVALID (table not symmetric, a constant out of range, ntypes above
 * max_materials, a type out of range). */
dem_status dem_set_materials(dem_system *s, int32_t ntypes, const double *table, const int32_t *type,
                             int32_t wall_type);

/* Largest speed max_i |v_i| of the current state (FP64 norm of the stored
 * velocities).  Synchronous. */
dem_status dem_max_speed(dem_system *s, double *vmax);

/* Sec. 5 runs its sample problem until the displacements of all particles
 * are below a set value; here a particle's displacement is read as
 * dt |v_i|, the step it would make at its current velocity.  Steps in chunks
 * of check_every (the last chunk shorter if max_steps is reached) and stops
 * after the first chunk at whose end dt * max_i |v_i| < threshold, or when
 * max_steps are done; *steps_done tells which.  Synchronous.  Errors:
 * DEM_E_INVALID (threshold < 0, check_every < 1, max_steps < 0), else as
 * dem_step. */
dem_status dem_run_to_rest(dem_system *s, double threshold, int64_t check_every, int64_t max_steps,
                           int64_t *steps_done);

/* Phase timing.  With enable != 0 every later dem_step brackets each of its
 * phases with HIP events on the system's stream; dem_profile_read waits for
 * the stream, returns the milliseconds spent in each phase summed over the
 * steps timed since the previous read (and their number), then clears them.
 * Phases: 0 kick-drift-hash of a call's first step (Steps 1-2; later steps
 * do it inside phase 5), 1 sort and cell starts (Step 3), 2 reorder
 * (Step 4), 3 contact detection over the neighbouring cells (Steps 5-6 and
 * 8) with, for the direct launch shape, the contact law of each owned
 * contact in the same kernel (Step 7), 4 the contact-law pass of the systems
 * swept by the other launch shapes (empty otherwise), 5 per-particle sums,
 * closing kick and the next step's kick-drift-hash.  With graph replay the
 * whole step after phase 0 is counted in phase 5.  At most
 * DEM_PROFILE_CAPACITY steps are timed between two reads. */
#define DEM_NUM_PHASES 6
#define DEM_PROFILE_CAPACITY 4096
dem_status dem_profile(dem_system *s, int enable);
dem_status dem_profile_read(dem_system *s, double ms[DEM_NUM_PHASES], int64_t *steps);

/* Capture one time step (Steps 2-8 and the closing kick) into two HIP
 * graphs, one per buffer parity, and replay them in dem_step from then on.
 * The stream given to dem_create must not be the NULL stream (graph capture
 * needs a created stream).  Phase timing then counts whole steps in phase 6.
 * Results are identical with and without graphs.  enable = 0 goes back to
 * plain launches. */
dem_status dem_use_graph(dem_system *s, int enable);

/* Wait for the system's stream; report any sticky error. */
dem_status dem_sync(dem_system *s);

/* Free the host handle (the workspace stays the caller's).  Waits for the
 * stream first. */
dem_status dem_destroy(dem_system *s);

const char *dem_status_string(dem_status st);

/* ------------------------------------------------------------------------
 * Batches: many independent systems of uneven size stepped together.  All
 * systems of a batch share one workspace, one stream and one set of kernel
 * launches per step (each kernel serves every system; no system waits for
 * another's launch), and must share the contact law and the precision; every
 * other parameter (box, walls, gravity, dt, material, cell) is per system.
 * A system's results do not depend on the other systems of its batch: they
 * are bitwise those of the same system created alone with dem_create.
 * Host arrays are the systems' arrays concatenated in system order; ids in
 * contact keys are local to a system. */
typedef struct dem_batch dem_batch;

/* Device bytes for systems k = 0..n_sys-1 of n[k] particles, parameters p[k]. */
dem_status dem_batch_workspace_bytes(int32_t n_sys, const dem_params *p, const int64_t *n, size_t *bytes);

/* Create a batch from the systems' host arrays, concatenated in system order
 * (each as dem_create would take it).  F0, T0 (sum(n) x 3, or both NULL) and
 * the tangential history restart the systems exactly: n_hist[k] keys of
 * system k (ids local to it) follow those of system k - 1 in hist_pairs
 * (2 each) and hist_dt (3 each); n_hist NULL for none.  Synchronous.  Errors
 * as dem_create, plus DEM_E_INVALID when the systems' laws or precisions
 * differ. */
dem_status dem_batch_create(int32_t n_sys, const dem_params *p, const int64_t *n, const double *x,
                            const double *v, const double *omega, const double *r, const double *F0,
                            const double *T0, const int64_t *n_hist, const int64_t *hist_pairs,
                            const double *hist_dt, void *workspace, size_t ws_bytes, void *hip_stream,
                            dem_batch **out);

/* dem_set_radii for every system of the batch: r holds sum(n) radii,
 * concatenated in system order.  Synchronous. */
dem_status dem_batch_set_radii(dem_batch *b, const double *r);

/* dem_set_materials for system k of the batch (type: its n[k] particles in
 * its own order); the stored forces of system k only are evaluated again.
 * Synchronous. */
dem_status dem_batch_set_materials(dem_batch *b, int32_t k, int32_t ntypes, const double *table,
                                   const int32_t *type, int32_t wall_type);

/* dem_max_speed of every system: vmax[k] for k = 0..n_sys-1.  Synchronous. */
dem_status dem_batch_max_speed(dem_batch *b, double *vmax);

/* Advance system k by steps[k] >= 0 steps (0: it does not move).  The batch
 * runs max(steps) steps; a system that has done its steps stays unchanged
 * (state and history) while the others go on.  Asynchronous. */
dem_status dem_batch_step(dem_batch *b, const int64_t *steps);

/* State of system k (0 <= k < n_sys) as dem_read_state: its n[k] particles
 * in its own original order.  Synchronous.  Errors: DEM_E_INVALID for k out
 * of range, else the sticky error. */
dem_status dem_batch_read_state(dem_batch *b, int32_t k, double *x, double *v, double *omega, double *F,
                                double *T);
/* Committed history of system k as dem_read_contacts (keys local to it). */
dem_status dem_batch_read_contacts(dem_batch *b, int32_t k, int64_t cap, int64_t *n_out, int64_t *pairs,
                                   double *delta_t);
/* Diagnostics of every system: out[10 * k + j] as dem_diagnostics. */
dem_status dem_batch_diagnostics(dem_batch *b, double *out);
/* As dem_use_graph, dem_profile, dem_profile_read, dem_sync and dem_destroy,
 * for the whole batch (phases summed over all its systems). */
dem_status dem_batch_use_graph(dem_batch *b, int enable);
dem_status dem_batch_profile(dem_batch *b, int enable);
dem_status dem_batch_profile_read(dem_batch *b, double ms[DEM_NUM_PHASES], int64_t *steps);
dem_status dem_batch_sync(dem_batch *b);
dem_status dem_batch_destroy(dem_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* DEM_H */
