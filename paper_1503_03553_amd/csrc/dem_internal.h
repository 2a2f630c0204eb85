// Internal definitions shared by the HIP kernels and the host runtime of libdem.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/dem.h"

namespace dem {

constexpr int TILE = 128;                 // particles per force workgroup (2 waves)
constexpr int DTILE = TILE;               // particles per detect workgroup; also the unit of
                                          // the contact list's regions
constexpr uint32_t FACE = 0xFFFFFFF0u;    // partner code of box face f is FACE + f
constexpr int MAXMAT = 8;
constexpr int SORT_THREADS = 256;
constexpr int SORT_ITEMS = 8;
constexpr int SORT_TILE = SORT_THREADS * SORT_ITEMS;

// device error bits
constexpr uint32_t ERR_CAPACITY = 1u;     // contact table too small for this step
constexpr uint32_t ERR_ROW = 2u;          // a particle has more contacts than the row buffer
constexpr uint32_t ERR_NONFINITE = 4u;    // NaN / Inf in a force or the new state
constexpr uint32_t ERR_MOVERS = 8u;       // more particles changed cell than the merge sort takes

// Particles that may change cell in one step for the merge sort; beyond
// this the step is redone with the radix sort.
constexpr uint32_t MAX_MOVERS = 8192;

// Per material-pair constants of the contact law (section 2), computed on the
// host in FP64 and kept in device memory.
struct MatTable {
    double kn_pref[MAXMAT * MAXMAT];  // k_n = kn_pref sqrt(r*)
    double kt_pref[MAXMAT * MAXMAT];  // k_t = kt_pref sqrt(r* dn)
    double alpha[MAXMAT * MAXMAT];    // damping prefactor alpha(eps_ij)
    double mu[MAXMAT * MAXMAT];       // sliding friction mu_ij
    double mass_pref[MAXMAT];         // m = mass_pref r^3  (rho 4/3 pi)
};

// Box, grid and step constants, passed by value to every kernel.
struct Geo {
    double lo[3], hi[3], L[3];
    double inv_cell[3];
    double cw[3];           // cell widths L / nc
    double reach;           // largest radius of the particles the cell stencil pairs
                            // (all, or those up to rcut) plus a rounding margin: a
                            // partner of particle i is within r_i + reach of it
    double reach_big;       // largest radius of the job plus the margin (wide scan)
    double inv_L[3];        // 1 / L, for the minimum-image choice
    int nc[3];
    uint32_t walls, periodic;
    int le;                 // Lees-Edwards shear active
    float rcut;             // two-level contact search: particles of a larger radius
                            // ("big") pair through the wide scan; >= every radius
                            // when the job has none
    int nbig;               // whether the job has big particles
    int key_bits;           // bits of the cell key
    int xbits;              // bits of its x part (the fastest-varying index)
    double g[3];
    double dt;
    double le_shift;        // image offset along x at the start of the next step
    double le_shift_next;   // at its end (used when wrapping); both advanced by the
                            // end-of-step kernel
    double le_dv;           // shear_rate * L_y: image velocity along x
};

// One simulation of a pool (device-resident).  Its particles occupy the
// tile-aligned positions [p0, p0 + n) (the rest of its last tile are inactive
// "ghost" slots), its cell bounds start at cell_base, its materials are
// MatTable number `mat`.  Time, remaining steps, shear offsets and status
// advance on the device, in the end-of-step kernel only: within the other
// kernels of a step the descriptor is read-only.
constexpr uint32_t NO_JOB = 0xFFFFFFFFu;
constexpr uint32_t JOB_ACTIVE = 0u, JOB_DONE = 1u, JOB_FAILED = 2u;
struct Job {
    Geo g;
    double t;                      // simulation time at the start of the next step
    float margin;                  // FP32 pre-filter margin of the contact search
    uint32_t p0, n;
    uint32_t cell_base;
    uint32_t mat;
    uint32_t status;               // JOB_*
    uint32_t steps_left;
    uint32_t nxw;                  // extra walls of the job
    unsigned long long steps_done;
    const dem_wall* xw;            // its extra walls (device memory)
};

// Device-side status word (one per pool).
struct Status {
    uint32_t err;
    uint32_t need;          // largest tile contact count seen when a tile overflowed
    unsigned long long steps_done;
    uint32_t movers;        // particles whose cell key changed in the current step
    uint32_t pad;
};

// Running counters of one workgroup (one slot per tile, so no two
// workgroups ever update the same word): contacts written, contacts that found
// their history, contacts of the step before.
struct TileStats {
    unsigned long long m, matched, old;      // sums over completed steps
    uint32_t m_step, matched_step, old_step; // the step in progress (folded in by
    uint32_t pad;                            // the reorder kernel, so a redone step
};                                           // counts once)

// Particle state: position + (radius bits | pid << 32) in one 32-byte
// record, velocity and angular velocity in three 16-byte planes
// (vx,vy) (vz,wx) (wy,wz), and a material byte.  Two such buffers alternate:
// a step reads one through the permutation `perm` (sorted position ->
// buffer position) and writes the other in its own sorted order.
struct State {
    double4* xr;
    double2* vw;   // 3 planes of n
    uint8_t* mat;  // may be null (one material)
};

// The records the contact search reads, in the sorted order of the step:
// the FP64 position record and its compact FP32 form ((x, y, z) - lo and the
// radius; NaN coordinates beyond 3 box lengths).
// The sorted order of a step: the contact search's FP32 records in sorted
// order, and the permutation into the state buffer it is paired with, whose
// FP64 records (position, radius, id) serve every sorted position through it.
struct Sorted {
    const double4* xr;   // the paired state buffer's records (read through perm)
    uint32_t* perm;      // sorted position -> position in that state buffer
    float4* xf;          // FP32 records (x - lo, y - lo, z - lo, r), sorted order
};

__host__ __device__ inline uint64_t pack_meta(float r, uint32_t pid) {
    union { float f; uint32_t u; } c;
    c.f = r;
    return (uint64_t)c.u | ((uint64_t)pid << 32);
}

}  // namespace dem

// Launch wrappers (dem_kernels.hip).  `ntiles` tiles of TILE positions are
// processed; tile T belongs to job tile_job[T] (NO_JOB for a free tile) and
// carries the high key bits tile_key[T] of its segment; `ns` is the position
// capacity (the plane stride of the velocity and force arrays).
namespace dem {
struct PoolView {
    const Job* jobs;
    uint32_t* job_fail;            // per job: set on a non-finite force or state
    const uint32_t* tile_job;
    const uint32_t* tile_key;
    uint32_t ntiles;
    uint32_t ns;
    uint32_t lmask;                // local key bits: (1 << local bits) - 1
    const MatTable* mats;
    TileStats* ts;
    Status* st;
    bool any_periodic;
};
// FP32 pre-filter margin of the contact search for a box of this geometry.
float detect_margin(const Geo& G);
void launch_detect(const PoolView& P, int kmax, const Sorted& S, const uint2* cells, uint2* rows,
                   uint32_t* col_j, uint32_t slots, hipStream_t s);
// The force kernel writes the sort's input.  With `movers` non-null (the
// merge sort) that is the key of every position before the step (`oldkeys`)
// and (new key, position) of the particles whose key changed, appended to
// `movers` (at most MAX_MOVERS); otherwise (the radix sort) the new key and
// index of every position (`keys`, `vals`), and the kernel empties the
// bounds of the old cells.
// X: the state the step reads (through perm), Y: the state it writes (in
// sorted order); S: the sorted order (FP32 records, and X's records through
// its permutation).
void launch_force(const PoolView& P, bool fp64, const Sorted& S, const State& X, const State& Y,
                  const uint2* rows, const uint32_t* col_j, const uint2* rows_old,
                  const uint32_t* perm,
                  const uint32_t* tab_pid_old, const double* tab_dt_old, uint32_t* tab_pid_new,
                  double* tab_dt_new, uint64_t cap, uint2* cells, uint32_t* keys, uint32_t* vals,
                  void* fo, uint32_t* oldkeys, uint2* movers, hipStream_t s);
// Stable sort of the n = ntiles * TILE keys by merging the few particles
// that changed cell into the unchanged ones, which are still in key order;
// the result (keys_s, vals_s) equals the radix sort's.
// The fused single loop (detect and force in one kernel), then the clearing
// of the old cell bounds.
void launch_fused(const PoolView& P, bool fp64, const Sorted& S, const State& X, const State& Y,
                  uint2* rows, uint32_t* col_j, const uint2* rows_old, const uint32_t* perm,
                  const uint32_t* tab_pid_old, const double* tab_dt_old, uint32_t* tab_pid_new,
                  double* tab_dt_new, uint64_t cap, uint32_t slots, uint2* cells, uint32_t* keys,
                  uint32_t* vals, void* fo, uint32_t* oldkeys, uint2* movers, hipStream_t s);
// The action-reaction variant of the force step: pair forces of owned
// pairs, then per-particle sums and the end of the step.
void launch_action_reaction(const PoolView& P, bool fp64, const Sorted& S, const State& X,
                            const State& Y, const uint2* rows, const uint32_t* col_j,
                            const uint2* rows_old, const uint32_t* perm,
                            const uint32_t* tab_pid_old, const double* tab_dt_old,
                            uint32_t* tab_pid_new, double* tab_dt_new, uint64_t cap, void* pf,
                            uint2* cells, uint32_t* keys, uint32_t* vals, void* fo,
                            uint32_t* oldkeys, uint2* movers, hipStream_t s);
// The split as the paper has it: each particle's thread runs over its own
// contacts (no compaction across the workgroup).
void launch_force_thread(const PoolView& P, bool fp64, const Sorted& S, const State& X,
                         const State& Y, const uint2* rows, const uint32_t* col_j,
                         const uint2* rows_old, const uint32_t* perm, const uint32_t* tab_pid_old,
                         const double* tab_dt_old, uint32_t* tab_pid_new, double* tab_dt_new,
                         uint64_t cap, uint2* cells, uint32_t* keys, uint32_t* vals, void* fo,
                         uint32_t* oldkeys, uint2* movers, hipStream_t s);
// Contact search testing each pair once (the upper half of each particle's
// cell stencil), appending (position, partner id) to both particles'
// adjacency lists: slot k of particle p at adj[k * P.ns + p], kmax slots
// (8, 16 or 32; adj holds kmax * P.ns entries), deg[p] the list length (zero
// on entry; launch_force_half reads and resets it).
void launch_detect_half(const PoolView& P, int kmax, const Sorted& S, const uint2* cells,
                        uint32_t* deg, uint2* adj, hipStream_t s);
// The force kernel over the lists of launch_detect_half: writes the rows and
// partner list of the step (rows, col_j with `slots` entries per particle of
// a tile's region) from the lists, then runs as launch_force.
void launch_force_half(const PoolView& P, bool fp64, int kmax, const Sorted& S, const State& X,
                       const State& Y, uint32_t* deg, const uint2* adj, uint2* rows,
                       uint32_t* col_j, uint32_t slots, const uint2* rows_old,
                       const uint32_t* perm, const uint32_t* tab_pid_old,
                       const double* tab_dt_old, uint32_t* tab_pid_new, double* tab_dt_new,
                       uint64_t cap, uint2* cells, uint32_t* keys, uint32_t* vals, void* fo,
                       uint32_t* oldkeys, uint2* movers, hipStream_t s);
// The merge sort: the sorted keys (keys_s) and, placed directly at their
// new positions, the FP32 records S.xf of the state Y just written and the
// permutation perm (new sorted position -> position in Y).  S and perm are
// the buffers of the next step, not those this step read.  It also empties the cell bounds of the movers' old cells (the force
// kernel leaves them in place with this sort).
// It also ends the step for the `njobs` job descriptors P.jobs: each is
// written, advanced (time, steps, status) or unchanged, to jobs_next, the
// descriptors the next step reads.
void launch_merge_sort(const PoolView& P, const uint32_t* oldkeys, const uint2* movers,
                       unsigned long long* mk, uint32_t* mp, uint32_t* keys_s, const State& Y,
                       const Sorted& S, uint32_t* perm, uint2* cells, Job* jobs_next,
                       uint32_t njobs, hipStream_t s);
// Sorts (keys, vals) by the low `bits` bits of keys; the result ends in
// (keys_out, vals_out).  tmp buffers are the ping-pong partners.
void launch_radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* keys_tmp, uint32_t* vals_tmp,
                       uint32_t n, int bits, uint32_t* tile_hist, uint32_t* digit_tot,
                       uint32_t** keys_out, uint32_t** vals_out, const Status* st, hipStream_t s);
// After the sort: with `gather` (the radix sort) the permutation (new
// sorted position -> position in Y) and the FP32 records gathered from Y
// into the next step's buffers S.xf and perm; the cell bounds;
// the step's count.  With `gather` the step then ends for the `njobs` job
// descriptors P.jobs, written to jobs_next (the merge sort does this itself).
void launch_reorder(const PoolView& P, Job* jobs_next, uint32_t njobs, bool gather,
                    const uint32_t* keys_s, const uint32_t* vals_s, const State& Y,
                    const Sorted& S, uint32_t* perm, uint2* cells, hipStream_t s);
// Replaces the radii of the positions [p0, p0 + n) of one job (rnew in
// particle-id order) in the state X the next step reads and in the FP32
// records of its sorted order S.
void launch_set_radii(uint32_t p0, uint32_t n, const float* rnew, const State& X, const Sorted& S,
                      hipStream_t s);
// Rewrites the cell bounds of the current order from its positions (S).
void launch_rebuild_cells(const PoolView& P, const Sorted& S, uint2* cells, hipStream_t s);
size_t sort_hist_words(uint32_t n);
// Shear offset of the image along x at time t: D(t) = (shear_rate L_y t) mod L_x.
double le_offset(const Geo& G, double t);
}  // namespace dem
