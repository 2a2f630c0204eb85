/*
 * dem.h -- C ABI of the MI355X DEM force-step library (libdem.so).
 *
 * The library advances spheres under the contact law of Nakahara &
 * Washizawa, "Accelerating DEM simulations on GPUs by reducing the impact of
 * warp divergences" (arXiv:1503.03553), section 2: Hertz normal force
 * k_n dn^(3/2), Mindlin tangential stiffness k_t(dn), damping
 * eta = alpha(eps) sqrt(m* k_n sqrt(dn)), tangential displacement history
 * (Eq. 3) carried across steps, sliding cap (Eq. 4) and torque r (n x F).
 * Its calls follow the paper's problem statement (section 4.2, kernel list):
 * the host creates the initial configuration, sends it to the GPU once, and
 * then only asks the GPU to advance it.
 *
 * Conventions common to every call
 *  - Units are SI.  Arrays are interleaved xyz ((n,3) row-major) unless
 *    stated otherwise.
 *  - Particle identity: the input index is the particle id (pid).  Every
 *    output is returned in pid order, although the device keeps particles in
 *    cell order internally.
 *  - Ownership: the caller owns every host buffer; the library copies what it
 *    needs and never keeps a caller pointer after a call returns.  A
 *    dem_sim or dem_pool owns its device memory and frees it on destruction,
 *    unless the caller lent it a device arena at creation: then every device
 *    buffer is carved from that arena, which the caller keeps owning (it
 *    must outlive the handle and is never freed by the library).
 *  - Errors: every call returns a dem_status; nothing is thrown across the
 *    ABI.  dem_step only enqueues work; a condition found on the device
 *    (contact capacity, non-finite state) is reported by the next blocking
 *    call (dem_sync, dem_get_*), after which the state is that of the last
 *    step that completed.  Capacity overflow is handled inside the library
 *    (it grows the contact table and redoes the step) and only surfaces as
 *    DEM_ECAPACITY when memory cannot be grown.
 *  - Threading: one host thread at a time per handle.  Calls on different
 *    handles are independent.
 *  - Box faces ("walls") are the six faces of the box [lo, hi) as planes,
 *    with the contact law of a sphere of infinite radius and mass made of the
 *    particle's own material (section 3.3: forces between a particle and a
 *    wall are computed like those between particles).  In contact lists a
 *    face f is partner id DEM_FACE_ID + f, f = 2 * axis + (0 low, 1 high).
 */
#ifndef DEM_H
#define DEM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dem_sim dem_sim; /* opaque, owned by the library */

typedef enum {
    DEM_OK = 0,
    DEM_EINVAL = -1,      /* a bad argument; nothing was changed */
    DEM_ENOMEM = -2,      /* device or host allocation failed */
    DEM_ECAPACITY = -3,   /* contact table could not be grown */
    DEM_ENONFINITE = -4,  /* a force or state component became NaN/Inf */
    DEM_EDEVICE = -5,     /* a HIP runtime error */
    DEM_EBUSY = -6,       /* a pool has no room (particles, cells, job slots or key
                             bits) for this job now; nothing was changed */
    DEM_ESCRATCH = -7     /* dem_create_static: the simulation needs more device
                             memory than the static scratch holds */
} dem_status;

typedef enum {
    DEM_PREC_FP64 = 0,  /* every operation in FP64 */
    DEM_PREC_MIXED = 1  /* contact normal, velocities, stiffnesses and forces in
                           FP32; overlap, tangential displacement history,
                           positions, velocities and angular velocities in FP64 */
} dem_precision;

#define DEM_MAX_MATERIALS 8
#define DEM_FACE_ID 0xFFFFFFF0u

/* One material (section 2: E Young's modulus, sigma Poisson ratio, G shear
 * modulus, eps restitution coefficient, mu_D sliding friction coefficient).
 * A pair of materials uses the means of their restitution and friction. */
typedef struct {
    double E, poisson, G, density, restitution, mu;
} dem_material;

/* A static wall inside the box besides its faces (section 3.3, item 5 of the
 * changes to the sample code: rectangles and straight lines; section 4.2,
 * kernel list: "CollideRectangle", "CollideLine"): kind DEM_WALL_RECT is the closed
 * rectangle p + s u + t v (u and v orthogonal and non-zero), kind
 * DEM_WALL_SEGMENT the closed segment p + s u; s, t in [0, 1], lengths in
 * metres.  Like a box face it is a body of infinite radius and mass with the
 * particle's material.  The contact point is the wall's point closest to
 * the particle centre; the particle touches the wall when that point is
 * nearer than its radius (a centre exactly on a segment makes no contact; a
 * centre exactly on a rectangle takes the normal u x v).  Extra wall k has
 * partner id DEM_FACE_ID + 6 + k in the contact history. */
typedef struct {
    int32_t kind;
    uint32_t reserved;
    double p[3], u[3], v[3];
} dem_wall;
#define DEM_WALL_RECT 0
#define DEM_WALL_SEGMENT 1
#define DEM_MAX_WALLS 10

typedef struct {
    double lo[3], hi[3]; /* box [m] */
    uint32_t walls;      /* bit 2a: low face of axis a is a wall; bit 2a+1: high face */
    uint32_t periodic;   /* bit a: axis a periodic (no wall on it) */
    double gravity[3];   /* [m/s^2], added as m g ("ForceGravity") */
    double shear_rate;   /* Lees-Edwards shear d(v_x)/dy [1/s]; needs x and y periodic; 0 = off */
    double dt;           /* time step [s]; 0 = t_c/50, t_c the undamped head-on contact
                            time of two spheres of the smallest radius at 0.1 m/s */
    double time;         /* simulation time of the initial state [s] (shear offset) */
    int32_t precision;   /* dem_precision */
    int32_t kn_form;     /* 0: k_n with (2 - sigma^2)/E as printed in section 2;
                            1: textbook Hertz (1 - sigma^2)/E */
    double cell_size;    /* [m]; 0 = automatic: twice the radius cut of the two-level
                            search (radius_cut below) with the default search, the
                            largest contact distance 2 r_max with the full one.  A
                            given size must be >= 2 r_max (one-level search). */
    uint64_t max_contacts; /* initial contact-table capacity; 0 = automatic */
    uint32_t flags;        /* DEM_FLAG_* */
    uint32_t n_extra_walls;          /* entries of extra_walls, at most DEM_MAX_WALLS */
    const dem_wall *extra_walls;     /* copied at creation; may be null when none */
    double radius_cut;   /* [m] two-level contact search (default search, automatic
                            cells): particles above this radius scan a two-cell
                            stencil themselves and the cells are sized for twice
                            the cut; raised to r_max / 2 if lower, r_max or more
                            means one level.  0 = automatic: one level below volume
                            fraction 0.3, else the radius exceeded by about 0.1 %
                            of the particles */
} dem_params;

#define DEM_FLAG_NO_FORCE_OUTPUT 1u /* do not store per-particle F, T each step */
#define DEM_FLAG_RADIX_SORT 2u      /* sort all keys every step (LSD radix sort) instead of
                                       merging the particles that changed cell; same
                                       results, for comparison */
#define DEM_FLAG_FUSED 4u           /* ablation of the split of section 3.4: one kernel
                                       whose lane per particle runs the contact law as
                                       soon as it finds a contact (Algorithm 1 before
                                       the split).  Same contact set; the per-particle
                                       sums follow the order the contacts were found
                                       instead of ascending partner id */
#define DEM_FLAG_ACTION_REACTION 8u /* each particle pair's force computed once, by the
                                       particle with the lower id, and applied with
                                       opposite signs to both (the scheme section 3.3
                                       avoids); sums stay in ascending partner id.  The
                                       history keeps one displacement per pair;
                                       dem_get_contacts reports the other direction as
                                       its negative.  Not with DEM_FLAG_FUSED */
#define DEM_FLAG_THREAD_SPLIT 16u   /* the split as section 3.4 has it: each particle's
                                       thread runs the contact law over the contacts
                                       its first loop found, with no compaction across
                                       the workgroup; same results as the default path.
                                       For comparison; at most one of DEM_FLAG_FUSED,
                                       DEM_FLAG_ACTION_REACTION and this flag */
#define DEM_FLAG_FULL_DETECT 32u    /* contact search as Algorithm 1 (section 3.3) has
                                       it: each particle scans its whole 27-cell stencil
                                       and writes its own row.  The default scans the upper half of the
                                       stencil, so each pair is tested once, and enters
                                       each contact in both particles' rows; both give
                                       the same rows.  DEM_FLAG_FUSED,
                                       DEM_FLAG_ACTION_REACTION and DEM_FLAG_THREAD_SPLIT
                                       always use the full search */

/* Diagnostics of a simulation (dem_get_info). */
typedef struct {
    uint64_t n;             /* particles */
    uint64_t steps_done;    /* completed steps since dem_create */
    double dt, time;        /* time step and current simulation time */
    uint64_t contacts;      /* directed contacts (including faces) in the last step */
    uint64_t capacity;      /* contact-table capacity */
    uint64_t regrows;       /* capacity regrowths so far */
    uint64_t sum_contacts;  /* sums over completed steps: contacts, */
    uint64_t sum_matched;   /*   contacts that carried history from the step before, */
    uint64_t sum_old;       /*   contacts of the step before */
    uint32_t cells[3];      /* cell grid */
    uint32_t key_bits;      /* bits of the cell key sorted each step */
    uint64_t device_bytes;  /* device memory held */
    double radius_cut;      /* two-level contact search: particles of a larger radius
                               scan a two-cell stencil themselves; the largest
                               radius when none do */
    uint64_t big;           /* particles above the radius cut */
} dem_info;

/*
 * Create a simulation and upload its initial state (section 4.2: the only
 * work of the CPU is to create the initial configuration and send it to the
 * GPU; section 2 names the state: positions, velocities, angular
 * velocities, radii and materials).
 *   params, mats[n_mats]   box, walls, gravity, time step, precision, materials
 *   n                      particles (0 allowed)
 *   x, v, w                (n,3) positions, velocities, angular velocities;
 *                          along a periodic axis positions must lie in [lo, hi]
 *   radius                 (n) radii; FP32 so that sums of two radii are exact in FP64
 *   mat_id                 (n) material index < n_mats, or NULL for all 0
 *   device_arena           NULL: the library allocates its device memory.
 *                          Otherwise device memory of arena_bytes bytes, aligned
 *                          to 256 bytes, lent by the caller (e.g. a torch uint8
 *                          tensor): every device buffer of the simulation is
 *                          carved from it.  arena_bytes must be at least
 *                          dem_footprint(params, n); room beyond that lets the
 *                          contact table grow (without room, growth fails with
 *                          DEM_ECAPACITY).  The arena must outlive the handle.
 *   stream                 hipStream_t to enqueue on, or NULL for the null stream
 * On success *out receives the handle.  Returns DEM_EINVAL for a bad box,
 * materials, radius, a position outside the box along a periodic axis, a
 * particle id space over 2^32 - 16, fewer than 3 cells along a periodic axis,
 * a wall on a periodic axis, or an arena that is misaligned or too small.
 */
dem_status dem_create(const dem_params *params, const dem_material *mats, uint32_t n_mats,
                      uint64_t n, const double *x, const double *v, const double *w,
                      const float *radius, const uint16_t *mat_id, void *device_arena,
                      uint64_t arena_bytes, void *stream, dem_sim **out);

/*
 * dem_create without any device allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops that must not
 * call hipMalloc, harnesses that forbid it).  Arguments and results are those
 * of dem_create; instead of allocating, or borrowing a caller's arena, the
 * simulation lives in a static scratch array of DEM_STATIC_BYTES that the
 * library reserves on each device it runs on (held until the process ends).
 * Neither this call nor any later call on the handle allocates device memory:
 * contact-table growth beyond the scratch's spare room fails with
 * DEM_ECAPACITY, as with a lent arena.
 *  - DEM_ESCRATCH: dem_footprint(params, n) exceeds DEM_STATIC_BYTES
 *    (about 75,000 particles with the default contact table); nothing was
 *    created.
 *  - DEM_EBUSY: a simulation made by this call still lives on the current
 *    device (one per device at a time: they would share the array); destroy
 *    it first.  Simulations on different devices are independent.
 * The scratch keeps the contents of the simulation that used it last; every
 * buffer that must start at zero is cleared at creation.  Creation and use
 * from several threads must not overlap on one device.
 */
#define DEM_STATIC_BYTES (64ull << 20)
dem_status dem_create_static(const dem_params *params, const dem_material *mats, uint32_t n_mats,
                             uint64_t n, const double *x, const double *v, const double *w,
                             const float *radius, const uint16_t *mat_id, void *stream,
                             dem_sim **out);

/*
 * Enqueue nsteps time steps on the simulation's stream and return (section
 * 4.2: the CPU only calls the GPU kernels again and again; section 3.4: the
 * force loop split into a contact search and a force loop).  One step is:
 * contact search (by default over the upper half of the 27 cells around
 * each particle, each pair tested once and entered in both particles'
 * lists, the few particles above the radius cut scanning a two-cell stencil
 * themselves; the full 27-cell scan of section 3.3 with DEM_FLAG_FULL_DETECT),
 * contact history match, contact law (Eq. 1-4, torque), per-particle sums
 * with gravity, semi-implicit Euler integration of velocity, position and
 * angular velocity, cell hashing, the sort by cell key (merge of the
 * particles that changed cell, radix sort as fallback) and the reorder into
 * cell order.
 */
dem_status dem_step(dem_sim *sim, uint32_t nsteps);

/* Wait for the enqueued steps (section 4.2: the host's loop over the GPU
 * kernels); handles capacity regrowth and redoes an abandoned step; reports
 * device errors. */
dem_status dem_sync(dem_sim *sim);

/*
 * Copy the current state to host buffers in pid order (blocking): the
 * position, velocity and angular velocity the "Integrate" kernel updates
 * (section 4.2) and the force and torque of Eq. (1) and the torque line of
 * section 2 summed over each particle's contacts, with m g ("ForceGravity").
 * Any pointer may be NULL to skip it.  F, T are those used by the last
 * completed step (zero before the first step or with
 * DEM_FLAG_NO_FORCE_OUTPUT).
 */
dem_status dem_get_state(dem_sim *sim, double *x, double *v, double *w, double *F, double *T);

/*
 * Copy the contact history to host buffers (blocking): the pair-wise
 * tangential displacement of Eq. (3), which section 4.2 stores like a sparse
 * matrix ("InitializeContactIDs" keeps only the pairs in contact).  For every
 * directed contact (i, j) of the last completed step, sorted by (i, j), its
 * displacement dt_xyz (3 doubles).  j is a pid or DEM_FACE_ID + f.  At most
 * cap entries are written; *m receives the total count (call with cap = 0 to
 * size the buffers).
 */
dem_status dem_get_contacts(dem_sim *sim, uint64_t cap, uint32_t *i, uint32_t *j, double *dt_xyz,
                            uint64_t *m);

/*
 * Replace the contact history used by the next step (the sparse matrix of
 * tangential displacements of section 4.2; for tests and resume).  Entries
 * need not be sorted; duplicate (i, j) pairs are rejected.
 */
dem_status dem_set_contacts(dem_sim *sim, uint64_t m, const uint32_t *i, const uint32_t *j,
                            const double *dt_xyz);

/* Replace positions, velocities, angular velocities (pid order; the state of
 * section 2 that section 4.2's initial configuration sets); the contact
 * history is kept.  Positions must lie in [lo, hi] along periodic axes. */
dem_status dem_set_state(dem_sim *sim, const double *x, const double *v, const double *w);

/* Replace the radii (pid order; the particle sizes of section 2's contact
 * law), keeping positions, velocities, angular velocities and the contact
 * history; masses and moments of inertia follow the new radii, the time step
 * stays.  Used to grow a packing by inflating its particles.  DEM_EINVAL for
 * a radius that is not finite and positive, or when twice the largest radius
 * exceeds a cell width of the simulation's grid (create it with a cell_size
 * for the largest radius it will reach). */
dem_status dem_set_radii(dem_sim *sim, const float *radius);

/* Diagnostics (blocking): step count, time, and the contact counts per step
 * (section 3.4: the number of contacts per particle sets the work of the
 * force loop). */
dem_status dem_get_info(dem_sim *sim, dem_info *info);

/* Free the simulation and the device memory it allocated (a lent arena is
 * left to its owner).  NULL is ignored.  Housekeeping of the handle; the
 * paper has no counterpart. */
void dem_destroy(dem_sim *sim);

/* A static string for a status code (housekeeping; no counterpart in the
 * paper). */
const char *dem_status_str(dem_status s);

/* Device bytes a simulation of n particles with these parameters needs at
 * creation (contact table at its automatic initial capacity): the size of
 * the arena dem_create needs (section 4.2: every array of the method lives
 * on the GPU). */
uint64_t dem_footprint(const dem_params *params, uint64_t n);

/*
 * Kernel timing (section 5.2 times each kernel of the step).  dem_profile(sim,
 * 1) makes every following dem_step record HIP events around each phase on
 * the simulation's stream; dem_profile_read waits and returns, per phase,
 * the summed milliseconds and the launch count since the last read (then
 * resets).  Phases: 0 detect, 1 force (history match, contact law, sums,
 * integration, hashing), 2 sort, 3 reorder.
 */
#define DEM_NPHASE 4
dem_status dem_profile(dem_sim *sim, int enable);
dem_status dem_profile_read(dem_sim *sim, double *ms, uint64_t *launches);

/* ===================================================================== pool
 *
 * A pool advances many independent simulations ("jobs") of uneven sizes with
 * one set of kernel launches per step: the data-parallel decomposition of
 * section 3.3 and 4.2 (one thread per particle, the step as a fixed sequence
 * of kernels over all particles) applied across jobs instead of within one.
 * Each job occupies whole 128-particle tiles, has its own box, walls,
 * gravity, shear, time step, materials and contact history, and is bitwise
 * independent of its neighbours: a job gives the same results alone
 * (dem_create) as in any mix.  All jobs of a pool share one precision.  Jobs
 * run for a fixed number of steps; a finished or failed job stays frozen in
 * the pool until removed.  Admission (dem_pool_add) and removal happen
 * between steps, so new jobs can join while others run (continuous
 * batching).  The paper runs one simulation at a time; the pool applies its
 * step unchanged to each job.
 */
typedef struct dem_pool dem_pool; /* opaque, owned by the library */

typedef struct {
    uint64_t max_particles;  /* particle positions (rounded up to 128-particle tiles);
                                0: the most that fit hbm_budget (see below) */
    uint64_t max_cells;      /* cell-table entries shared by all jobs' grids; with
                                max_particles = 0, 0 means 4 per position plus 4096
                                per job slot */
    uint32_t max_jobs;       /* job slots (with max_particles = 0, 0 means 256) */
    int32_t precision;       /* dem_precision of every job */
    uint32_t contact_slots;  /* initial contact slots per particle position; 0 = 8 */
    uint32_t flags;          /* DEM_FLAG_* */
    uint64_t hbm_budget;     /* device bytes the pool may take: with max_particles = 0
                                the capacities are the largest whose footprint fits
                                (the arena's size when 0 and an arena is lent);
                                otherwise a footprint above a non-zero budget is
                                DEM_EINVAL */
} dem_pool_params;

typedef enum { DEM_JOB_RUNNING = 0, DEM_JOB_DONE = 1, DEM_JOB_FAILED = 2 } dem_job_status;

typedef struct {
    int32_t status;       /* dem_job_status; FAILED = a non-finite force or state */
    uint32_t reserved;
    uint64_t n;           /* particles */
    uint64_t steps_done;  /* completed steps */
    uint64_t steps_left;  /* steps still to run */
    double time, dt;      /* simulation time and time step */
} dem_job_info;

/* Device bytes dem_pool_create allocates (or needs in a lent arena) for these
 * parameters (section 4.2: every array of the method lives on the GPU); 0 for
 * invalid parameters. */
uint64_t dem_pool_footprint(const dem_pool_params *pp);

/* Create an empty pool with all its device memory (no allocation happens in
 * later calls unless the contact table must grow).  device_arena and
 * arena_bytes as in dem_create (at least dem_pool_footprint(pp) bytes);
 * stream as in dem_create.  Section 4.2: the device holds everything; the
 * host only admits jobs and calls the kernels. */
dem_status dem_pool_create(const dem_pool_params *pp, void *device_arena, uint64_t arena_bytes,
                           void *stream, dem_pool **out);

/*
 * Admit one job that will run `steps` steps (1 .. 2^32 - 2): its initial
 * configuration is sent to the device as in dem_create (section 4.2).
 * Arguments are those of dem_create; params->precision must equal the
 * pool's, params->max_contacts and params->flags are ignored (the pool's
 * apply).  The upload is enqueued on the pool's stream.  On success *job
 * receives an id unique within the pool.  DEM_EBUSY: not enough contiguous
 * free tiles, cells or slots, or the pool's sort key would exceed 32 bits.
 */
dem_status dem_pool_add(dem_pool *pool, const dem_params *params, const dem_material *mats,
                        uint32_t n_mats, uint64_t n, const double *x, const double *v,
                        const double *w, const float *radius, const uint16_t *mat_id,
                        uint32_t steps, uint64_t *job);

/*
 * The host half of dem_pool_add, separately (section 4.2: creating the
 * initial configuration is the host's only work): dem_job_prepare validates
 * a job and places its particles in cell order (arguments as dem_pool_add;
 * no GPU call, safe to run on other threads while a pool steps);
 * dem_pool_add_prepared then admits it between steps (DEM_EBUSY leaves the
 * prepared job usable for a later try; any other outcome consumes it).
 * dem_job_prep_cells gives the cells it takes (0 once consumed), and
 * dem_job_prep_free releases it (NULL ignored).  The host copies of a
 * prepared job are owned by it until it is admitted.
 */
typedef struct dem_job_prep dem_job_prep; /* opaque */
dem_status dem_job_prepare(const dem_params *params, const dem_material *mats, uint32_t n_mats,
                           uint64_t n, const double *x, const double *v, const double *w,
                           const float *radius, const uint16_t *mat_id, dem_job_prep **out);
uint64_t dem_job_prep_cells(const dem_job_prep *prep);
dem_status dem_pool_add_prepared(dem_pool *pool, dem_job_prep *prep, uint32_t steps,
                                 uint64_t *job);
void dem_job_prep_free(dem_job_prep *prep);

/* Enqueue nsteps steps of every running job (finished jobs are skipped): the
 * step of dem_step (section 4.2 kernel list, section 3.4 split) over all
 * jobs at once. */
dem_status dem_pool_step(dem_pool *pool, uint32_t nsteps);

/* Wait for enqueued steps; capacity regrowth as in dem_sync.  A job's
 * non-finite failure is not a pool error: it shows as DEM_JOB_FAILED. */
dem_status dem_pool_sync(dem_pool *pool);

/* Wait, then write up to cap ids of jobs that finished or failed since the
 * last poll; *n_done receives the count written (host side of the serving
 * loop; no counterpart in the paper). */
dem_status dem_pool_poll(dem_pool *pool, uint64_t *done, uint32_t cap, uint32_t *n_done);

/* Status, step counts and time of a job (blocking). */
dem_status dem_pool_job_info(dem_pool *pool, uint64_t job, dem_job_info *info);

/* A job's state in pid order, as dem_get_state (blocking); NULL skips. */
dem_status dem_pool_get_state(dem_pool *pool, uint64_t job, double *x, double *v, double *w);

/* New radii of a job (pid order), as dem_set_radii (between steps). */
dem_status dem_pool_set_radii(dem_pool *pool, uint64_t job, const float *radius);

/* Free a job's tiles, cells and slot (between steps; enqueued in order). */
dem_status dem_pool_remove(dem_pool *pool, uint64_t job);

/* Room for the next job: the largest contiguous run of free particle
 * positions and of free cells, and the free job slots.  NULL skips.
 * Admission by device footprint (host side of the serving loop). */
dem_status dem_pool_capacity(dem_pool *pool, uint64_t *free_particles, uint64_t *free_cells,
                             uint32_t *free_jobs);

/* The most cells the grid of a job of n particles with these parameters and
 * largest radius rmax can get (what it may take of the pool's max_cells); 0
 * if the parameters are invalid.  Section 3.3: the cell-based search needs
 * cells at least as wide as the largest contact distance; with the two-level
 * search of the default (half) search, cells of twice a radius cut of at
 * least rmax / 2.  With dem_pool_capacity this tells whether a job fits
 * before its data is prepared. */
uint64_t dem_job_cells(const dem_params *params, uint64_t n, double rmax);

/* Kernel timing of the pool's steps, as dem_profile / dem_profile_read. */
dem_status dem_pool_profile(dem_pool *pool, int enable);
dem_status dem_pool_profile_read(dem_pool *pool, double *ms, uint64_t *launches);

/* Free the pool and the device memory it allocated (a lent arena is left to
 * its owner).  NULL is ignored. */
void dem_pool_destroy(dem_pool *pool);

#ifdef __cplusplus
}
#endif
#endif /* DEM_H */
