// Host runtime of libdem: validation, device memory, the job pool (several
// independent simulations advanced by the same kernel launches), the step
// pipeline with capacity regrowth, state and contact-history transfer, and
// the C ABI declared in include/dem.h.  A single simulation (dem_sim) is a
// pool holding one job.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <numeric>
#include <vector>

#include "../../include/dem.h"
#include "dem_internal.h"

using namespace dem;

namespace {

constexpr double PI = 3.14159265358979323846;
constexpr uint64_t MAX_ENTRIES = 0xFFFFFFF0ull;  // row starts and positions are 32-bit

// Damping prefactor alpha(eps) (section 2 defines eta = alpha(eps) sqrt(m* k_n
// sqrt(dn)) without giving alpha).  For the normal force k_n d^(3/2) + eta d',
// nondimensionalising the head-on collision leaves d'' = -d^(3/2) - alpha d^(1/4) d';
// alpha = -sqrt(5) ln(eps) / sqrt(ln^2 eps + pi^2) is the published closed form
// for which that collision ends with relative speed eps times the initial one.
double restitution_alpha(double eps) {
    if (eps >= 1.0) return 0.0;
    const double l = std::log(eps);
    return -std::sqrt(5.0) * l / std::sqrt(l * l + PI * PI);
}

// Duration of an undamped head-on Hertz contact at approach speed v0:
// (m*/k_n)^(2/5) v0^(-1/5) times 2 int_0^{(5/4)^(2/5)} ds / sqrt(1 - 4/5 s^(5/2)),
// which equals (4/5) (5/4)^(2/5) Gamma(2/5) Gamma(1/2) / Gamma(9/10).
double hertz_contact_time(double mstar, double kn, double v0) {
    const double c = 0.8 * std::pow(1.25, 0.4) * std::tgamma(0.4) * std::tgamma(0.5) / std::tgamma(0.9);
    return c * std::pow(mstar / kn, 0.4) * std::pow(v0, -0.2);
}

uint32_t spread2_host(uint32_t v) {
    v &= 0xFFFFu;
    v = (v | (v << 8)) & 0x00FF00FFu;
    v = (v | (v << 4)) & 0x0F0F0F0Fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}

struct Buf {
    void* p = nullptr;
    size_t bytes = 0;
    bool in_arena = false;  // carved from a borrowed arena: never passed to hipFree
};

// Phase boundaries of one step: phase p runs between events p and p + 1.
struct ProfEv {
    hipEvent_t e[DEM_NPHASE + 1];
};

struct Layout {
    int nc[3];
    double cell[3];
    int key_bits, xbits;
};

// One contiguous run of tiles (a job's segment or a free gap).
struct Seg {
    uint32_t start, len;
    int slot;  // job slot, -1 when free
};

struct HostJob {
    bool used = false;
    uint64_t id = 0;
    dem_params P{};
    std::vector<dem_material> mats;
    uint64_t n = 0;
    uint32_t tile0 = 0, ntiles = 0;
    uint32_t cell_base = 0, ncells = 0;
    Layout lay{};
    Geo geo{};
    bool multi_mat = false;
    bool reported = false;    // finished/failed status already returned by poll
    std::vector<float> r;
    std::vector<uint16_t> mat;
    std::vector<dem_wall> walls;  // extra walls (P.extra_walls is not kept)
    bool two_level = false;       // grid sized for the radius cut (half search)
};

uint64_t tiles_of(uint64_t n) { return (n + TILE - 1) / TILE; }

}  // namespace

struct dem_pool {
    hipStream_t stream = nullptr;
    // a borrowed device arena (caller memory): every device buffer is carved
    // from it in order; the library never frees it
    char* arena = nullptr;
    size_t arena_bytes = 0, arena_used = 0;
    bool fp64 = false;
    uint32_t flags = 0;
    int kmax = 8;                     // row buffer of the detect kernel (8, 16 or 32)
    uint32_t slots = 8;               // contact slots per position
    uint64_t cap = 0;                 // max_tiles * TILE * slots
    uint32_t max_tiles = 0, max_jobs = 0;
    uint64_t max_cells = 0;
    uint32_t hw_tiles = 0;            // tiles processed per step (high-water mark)
    int lb = 1;                       // local key bits
    bool any_periodic = false, any_multi_mat = false;
    std::vector<Seg> segs;            // tile segments in memory order
    std::vector<std::pair<uint64_t, uint64_t>> free_cells;  // (start, len)
    std::vector<HostJob> jobs;        // by slot
    uint64_t next_id = 1;
    int cur = 0;                      // table/rows buffer read as "old" by the next step
    std::deque<int> pending;          // buffer parity of each enqueued, unconfirmed step
    uint64_t steps_confirmed = 0;
    uint64_t regrows = 0;
    dem_status failed = DEM_OK;
    std::vector<std::vector<char>> staging;  // host buffers of uploads in flight
    std::vector<std::shared_ptr<void>> held; // host arrays moved in for uploads in flight
    // device memory
    std::vector<Buf> bufs;
    size_t device_bytes = 0;
    State S[2]{};                     // state buffers; S[cur] holds the current state
    // the sorted order a step reads (FP32 records, permutation into the
    // state buffer, whose FP64 records it reads through it), one per state
    // buffer: a step reads that of S[o] and writes that of S[w], so that an
    // abandoned step leaves the one it started from intact
    Sorted srt[2]{};
    uint2* cells = nullptr;
    uint2* rows[2] = {nullptr, nullptr};
    uint32_t* col_j = nullptr;
    uint32_t* tab_pid[2] = {nullptr, nullptr};
    double* tab_dt[2] = {nullptr, nullptr};
    uint32_t* prev[2] = {nullptr, nullptr};
    uint32_t *keys = nullptr, *vals = nullptr, *keys_t = nullptr, *vals_t = nullptr;
    uint32_t* tile_hist = nullptr;
    uint32_t* digit_tot = nullptr;
    uint32_t* oldkeys = nullptr;          // merge sort: keys before the step
    uint2* movers = nullptr;              //   (new key, position) of cell changers
    unsigned long long* mk = nullptr;     //   movers by (key, position)
    uint32_t* mp = nullptr;               //   movers by position
    uint32_t radix_left = 0;              // steps to take with the radix sort
    void* fo = nullptr;
    void* pf = nullptr;                   // action-reaction: pair F and n x F per entry
    uint32_t* deg = nullptr;              // half search: list length per particle
    uint2* adj = nullptr;                 //   and adjacency lists (adj_slots entries each)
    int adj_slots = 0;
    MatTable* mats = nullptr;
    // job descriptors, two buffers: a step reads jobs_d[o] (o: the state
    // buffer it reads) and its end writes jobs_d[w]; jobs_d[cur] holds those
    // the next step reads
    Job* jobs_d[2] = {nullptr, nullptr};
    dem_wall* walls_d = nullptr;          // DEM_MAX_WALLS extra walls per job slot
    uint32_t* job_fail = nullptr;
    uint32_t* tile_job = nullptr;
    uint32_t* tile_key = nullptr;
    TileStats* ts = nullptr;
    Status* st = nullptr;
    // profiling
    bool prof = false;
    std::vector<ProfEv> prof_ev;
    size_t prof_used = 0;
};

struct dem_sim {
    dem_pool* pool = nullptr;
    int slot = 0;
    int static_dev = -1;  // device whose static scratch holds it (dem_create_static), else -1
};

namespace {

dem_status hip_status(hipError_t e) {
    if (e == hipSuccess) return DEM_OK;
    if (e == hipErrorOutOfMemory) return DEM_ENOMEM;
    return DEM_EDEVICE;
}

#define HIPCHK(x)                                    \
    do {                                             \
        hipError_t e_ = (x);                         \
        if (e_ != hipSuccess) return hip_status(e_); \
    } while (0)

// Alignment of every buffer carved from an arena (and of the arena itself).
constexpr size_t ARENA_ALIGN = 256;

dem_status dalloc(dem_pool* s, size_t bytes, void** out) {
    void* p = nullptr;
    if (bytes == 0) bytes = 256;
    if (s->arena) {
        const size_t off = (s->arena_used + ARENA_ALIGN - 1) & ~(ARENA_ALIGN - 1);
        if (off > s->arena_bytes || bytes > s->arena_bytes - off) return DEM_ENOMEM;
        p = s->arena + off;
        s->arena_used = off + bytes;
        s->bufs.push_back({p, bytes, true});
    } else {
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return DEM_ENOMEM;
        }
        s->bufs.push_back({p, bytes, false});
    }
    s->device_bytes += bytes;
    *out = p;
    return DEM_OK;
}

// Free a device buffer.  A buffer carved from an arena returns its space
// only when it is the last one carved (growth beyond the arena's spare room
// then fails with DEM_ECAPACITY instead of allocating).
void dfree(dem_pool* s, void* p) {
    if (!p) return;
    for (size_t k = 0; k < s->bufs.size(); ++k)
        if (s->bufs[k].p == p) {
            const Buf b = s->bufs[k];
            s->device_bytes -= b.bytes;
            s->bufs.erase(s->bufs.begin() + k);
            if (b.in_arena) {
                if ((char*)b.p + b.bytes == s->arena + s->arena_used)
                    s->arena_used = (size_t)((char*)b.p - s->arena);
            } else {
                (void)hipFree(p);
            }
            return;
        }
}

template <typename T>
dem_status dalloc_t(dem_pool* s, size_t count, T** out) {
    void* p;
    dem_status r = dalloc(s, count * sizeof(T), &p);
    if (r == DEM_OK) *out = (T*)p;
    return r;
}

// Asynchronous upload whose host copy stays alive until the next sync.
dem_status upload(dem_pool* s, void* dst, const void* src, size_t bytes) {
    if (!bytes) return DEM_OK;
    s->staging.emplace_back((const char*)src, (const char*)src + bytes);
    HIPCHK(hipMemcpyAsync(dst, s->staging.back().data(), bytes, hipMemcpyHostToDevice, s->stream));
    return DEM_OK;
}

// Asynchronous upload of a host array that the pool takes over until the
// next sync (no copy).
template <typename T>
dem_status upload_vec(dem_pool* s, void* dst, std::vector<T>& v) {
    if (v.empty()) return DEM_OK;
    auto h = std::make_shared<std::vector<T>>(std::move(v));
    s->held.push_back(h);
    HIPCHK(hipMemcpyAsync(dst, h->data(), h->size() * sizeof(T), hipMemcpyHostToDevice, s->stream));
    return DEM_OK;
}

// Per-pair constants of the contact law.
void fill_mat_table(const dem_params& P, const std::vector<dem_material>& m, MatTable& T) {
    std::memset(&T, 0, sizeof(T));
    const int nm = (int)m.size();
    for (int a = 0; a < nm; ++a) {
        T.mass_pref[a] = m[a].density * (4.0 / 3.0) * PI;
        for (int b = 0; b < nm; ++b) {
            const double sa = m[a].poisson, sb = m[b].poisson;
            const double ca = (P.kn_form == 1) ? 1.0 - sa * sa : 2.0 - sa * sa;
            const double cb = (P.kn_form == 1) ? 1.0 - sb * sb : 2.0 - sb * sb;
            const int k = a * MAXMAT + b;
            T.kn_pref[k] = (4.0 / 3.0) / (ca / m[a].E + cb / m[b].E);
            T.kt_pref[k] = 8.0 / ((2.0 - sa) / m[a].G + (2.0 - sb) / m[b].G);
            T.alpha[k] = restitution_alpha(0.5 * (m[a].restitution + m[b].restitution));
            T.mu[k] = 0.5 * (m[a].mu + m[b].mu);
        }
    }
}

// Uniform grid whose cells are at least the largest contact distance wide
// along every axis, so that the 27 cells around a particle hold all its
// possible partners.  At most max(4 n, 4096) cells: in dilute boxes the cells
// grow instead.
dem_status plan_grid(const dem_params& P, double rmax, uint64_t n, Layout& out) {
    const double range = 2.0 * rmax;
    double want = P.cell_size > 0.0 ? P.cell_size : range;
    if (want < range) return DEM_EINVAL;
    const uint64_t limit = std::max<uint64_t>(4 * n, 4096);
    for (int iter = 0; iter < 2000; ++iter) {
        uint64_t prod = 1;
        for (int a = 0; a < 3; ++a) {
            const double L = P.hi[a] - P.lo[a];
            double c = std::floor(L / (want * 1.000001));
            if (c < 1) c = 1;
            if (c > 1024) c = 1024;
            out.nc[a] = (int)c;
            out.cell[a] = L / c;
            prod *= (uint64_t)c;
        }
        if (prod > limit) {
            want *= 1.02;
            continue;
        }
        for (int a = 0; a < 3; ++a)
            if (((P.periodic >> a) & 1u) && out.nc[a] < 3) return DEM_EINVAL;
        auto bits = [](int c) {
            int b = 0;
            while ((1 << b) < c) ++b;
            return b;
        };
        out.xbits = bits(out.nc[0]);
        out.key_bits = out.xbits + 2 * std::max(bits(out.nc[1]), bits(out.nc[2]));
        return DEM_OK;
    }
    return DEM_EINVAL;
}

bool finite3(const double* p) { return std::isfinite(p[0]) && std::isfinite(p[1]) && std::isfinite(p[2]); }

// Whether a position lies in [lo, hi] along every periodic axis.  The cell
// of a position outside would be clamped into a border cell, whose stencil
// need not hold the partners that touch the position's periodic image, so
// such input is rejected rather than wrapped silently.
bool in_periodic_box(const dem_params& P, const double* x) {
    for (int a = 0; a < 3; ++a)
        if (((P.periodic >> a) & 1u) && !(x[a] >= P.lo[a] && x[a] <= P.hi[a])) return false;
    return true;
}

// Radius cut of the two-level contact search, at least half the largest
// radius (so that the largest contact distance spans at most two cells of
// twice the cut); the largest radius itself means a one-level grid.  A
// cut given in the parameters is taken as it is.  Automatically: one level
// below volume fraction 0.3, where each particle has few candidates and the
// finer grid costs the force, sort and reorder kernels more than the search
// saves; from 0.3 on, the radius exceeded by about 0.1 % of the particles
// (measured on the 8M pack at 0.55: search 1456 -> 1156 us; a cut at 1 % or
// 2 % leaves more big particles, whose wide scans then cost more).
double radius_cut(const dem_params& P, const float* radius, uint64_t n, double rmax) {
    double rc = rmax;
    if (P.radius_cut > 0.0) {
        rc = P.radius_cut;
    } else {
        if (n < 64) return rmax;
        double vol = 1.0, vp = 0.0;
        for (int a = 0; a < 3; ++a) vol *= P.hi[a] - P.lo[a];
        for (uint64_t i = 0; i < n; ++i) {
            const double r = radius[i];
            vp += r * r * r;
        }
        if (!(4.18879020478639098 * vp >= 0.3 * vol)) return rmax;  // 4/3 pi
        std::vector<float> r(radius, radius + n);
        const uint64_t k = (uint64_t)(0.999 * (double)(n - 1));
        std::nth_element(r.begin(), r.begin() + (long)k, r.end());
        rc = r[k];
    }
    rc = std::max(rc, 0.5 * rmax);
    return rc >= rmax ? rmax : rc;
}

// Grid of a job: cells at least twice the radius cut when the two-level
// search applies (every periodic axis then needs 5 cells, so that the wide
// scan's two-cell stencil meets no cell twice), else twice the largest
// radius.  `used` receives the cut the grid supports (rmax for a one-level
// grid): the grid may come out coarser than asked (a cell-count limit), and
// the cut then grows with it.  Cells of twice the cut hold every pair of
// particles up to the cut, and since the cut is at least rmax / 2 the
// largest contact distance spans at most two cells.
dem_status plan_job_grid(const dem_params& P, double rmax, double rcut, uint64_t n,
                         Layout& lay, double& used) {
    used = rmax;
    if (rcut < rmax && P.cell_size == 0.0 && plan_grid(P, rcut, n, lay) == DEM_OK) {
        bool ok = true;
        double cmin = INFINITY;
        for (int a = 0; a < 3; ++a) {
            cmin = std::min(cmin, lay.cell[a]);
            if (((P.periodic >> a) & 1u) && lay.nc[a] < 5) ok = false;
        }
        const double cut = std::min(rmax, 0.5 * cmin / 1.000001);
        if (ok && cut < rmax) {
            used = cut;
            return DEM_OK;
        }
    }
    return plan_grid(P, rmax, n, lay);
}

// The radius cut as the kernels compare it (a float no larger than `used`)
// and the reaches of the two stencils.
void set_cut(Geo& G, double used, double rmax, double span) {
    float rc = (float)used;
    if ((double)rc > used) rc = std::nextafter(rc, 0.0f);
    if (used >= rmax) rc = (float)rmax;
    G.rcut = rc;
    G.nbig = used < rmax ? 1 : 0;
    G.reach = (used < rmax ? (double)rc : rmax) + 1e-9 * span;
    G.reach_big = rmax + 1e-9 * span;
}

dem_status validate(const dem_params* P, const dem_material* mats, uint32_t n_mats) {
    if (!P || !mats || n_mats < 1 || n_mats > DEM_MAX_MATERIALS) return DEM_EINVAL;
    for (int a = 0; a < 3; ++a) {
        if (!std::isfinite(P->lo[a]) || !std::isfinite(P->hi[a]) || !(P->hi[a] > P->lo[a]))
            return DEM_EINVAL;
        if (!std::isfinite(P->gravity[a])) return DEM_EINVAL;
        if (((P->periodic >> a) & 1u) && (P->walls & (3u << (2 * a)))) return DEM_EINVAL;
    }
    if (P->walls & ~0x3Fu) return DEM_EINVAL;
    if (P->periodic & ~7u) return DEM_EINVAL;
    if (!std::isfinite(P->shear_rate) || !std::isfinite(P->dt) || P->dt < 0.0) return DEM_EINVAL;
    if (!std::isfinite(P->time)) return DEM_EINVAL;
    if (P->shear_rate != 0.0 && (P->periodic & 3u) != 3u) return DEM_EINVAL;
    if (P->precision != DEM_PREC_FP64 && P->precision != DEM_PREC_MIXED) return DEM_EINVAL;
    if (P->kn_form != 0 && P->kn_form != 1) return DEM_EINVAL;
    if (!(P->cell_size >= 0.0) || !std::isfinite(P->cell_size)) return DEM_EINVAL;
    if (!(P->radius_cut >= 0.0) || !std::isfinite(P->radius_cut)) return DEM_EINVAL;
    if (P->n_extra_walls > DEM_MAX_WALLS || (P->n_extra_walls && !P->extra_walls)) return DEM_EINVAL;
    for (uint32_t k = 0; k < P->n_extra_walls; ++k) {
        const dem_wall& W = P->extra_walls[k];
        if (W.kind != DEM_WALL_RECT && W.kind != DEM_WALL_SEGMENT) return DEM_EINVAL;
        if (!finite3(W.p) || !finite3(W.u) || !finite3(W.v)) return DEM_EINVAL;
        const double uu = W.u[0] * W.u[0] + W.u[1] * W.u[1] + W.u[2] * W.u[2];
        if (!(uu > 0.0)) return DEM_EINVAL;
        if (W.kind == DEM_WALL_RECT) {
            const double vv = W.v[0] * W.v[0] + W.v[1] * W.v[1] + W.v[2] * W.v[2];
            const double uv = W.u[0] * W.v[0] + W.u[1] * W.v[1] + W.u[2] * W.v[2];
            if (!(vv > 0.0) || !(std::fabs(uv) <= 1e-12 * std::sqrt(uu * vv))) return DEM_EINVAL;
        }
    }
    for (uint32_t k = 0; k < n_mats; ++k) {
        const dem_material& m = mats[k];
        if (!(m.E > 0) || !(m.G > 0) || !(m.density > 0) || !std::isfinite(m.E) ||
            !std::isfinite(m.G) || !std::isfinite(m.density))
            return DEM_EINVAL;
        if (!(m.poisson > -1.0 && m.poisson < 0.5)) return DEM_EINVAL;
        if (!(m.restitution > 0.0 && m.restitution <= 1.0)) return DEM_EINVAL;
        if (!(m.mu >= 0.0) || !std::isfinite(m.mu)) return DEM_EINVAL;
    }
    return DEM_OK;
}

// ------------------------------------------------------------- pool memory
dem_status alloc_contacts(dem_pool* s, uint32_t slots, uint32_t** col, uint32_t** pid0,
                          uint32_t** pid1, double** dt0, double** dt1) {
    const uint64_t cap = (uint64_t)s->max_tiles * TILE * slots;
    *col = nullptr;
    *pid0 = *pid1 = nullptr;
    *dt0 = *dt1 = nullptr;
    if (cap > MAX_ENTRIES) return DEM_ECAPACITY;
    bool ok = dalloc_t(s, cap, col) == DEM_OK && dalloc_t(s, cap, pid0) == DEM_OK &&
              dalloc_t(s, cap, pid1) == DEM_OK && dalloc_t(s, 3 * cap, dt0) == DEM_OK &&
              dalloc_t(s, 3 * cap, dt1) == DEM_OK;
    if (!ok) {
        dfree(s, *col);
        dfree(s, *pid0);
        dfree(s, *pid1);
        dfree(s, *dt0);
        dfree(s, *dt1);
        return DEM_ENOMEM;
    }
    return DEM_OK;
}

// Whether a pool's contact search is the half search (the default for the
// plain force kernel; the force-path variants use the full search).
bool half_search(uint32_t flags) {
    return !(flags & (DEM_FLAG_FULL_DETECT | DEM_FLAG_FUSED | DEM_FLAG_ACTION_REACTION |
                      DEM_FLAG_THREAD_SPLIT));
}

uint64_t pool_bytes(uint64_t max_tiles, uint64_t max_cells, uint64_t max_jobs, bool fp64,
                    uint64_t slots, uint32_t flags) {
    const uint64_t np = max_tiles * TILE;
    uint64_t b = 0;
    b += 2 * np * (32 + 48 + 1);       // two state buffers
    b += 2 * np * 16;                  // FP32 records of the sorted order, two steps
    b += np * 2 * 8;                   // contact rows, two steps
    b += np * 7 * 4;                   // permutation (two), keys and values (two), keys before
    b += (uint64_t)MAX_MOVERS * 20;    // mover lists
    b += np * 6 * (fp64 ? 8 : 4);      // per-particle F, T
    b += max_cells * 8;                // cell bounds
    b += np * slots * (4 + 2 * 28);    // partner list and two history tables
    if (flags & DEM_FLAG_ACTION_REACTION) b += np * slots * 6 * (fp64 ? 8 : 4);  // pair forces
    if (half_search(flags)) b += np * (4 + 8 * 8);  // adjacency lists (8 slots; more in a clump)
    b += sort_hist_words((uint32_t)np) * 4 + 256 * 4;
    b += max_jobs * (sizeof(MatTable) + 2 * sizeof(Job) + 4 + DEM_MAX_WALLS * sizeof(dem_wall));
    b += max_tiles * (8 + sizeof(TileStats)) + sizeof(Status);
    b += 52 * ARENA_ALIGN;  // alignment of each buffer in an arena
    return b;
}

void destroy_pool(dem_pool* s) {
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    for (auto& b : s->bufs)
        if (!b.in_arena) (void)hipFree(b.p);
    s->bufs.clear();
    for (auto& pe : s->prof_ev)
        for (int q = 0; q <= DEM_NPHASE; ++q) (void)hipEventDestroy(pe.e[q]);
    delete s;
}

dem_status create_pool(uint64_t max_particles, uint64_t max_cells, uint32_t max_jobs, bool fp64,
                       uint32_t slots, uint32_t flags, void* arena, uint64_t arena_bytes,
                       void* stream, dem_pool** out) {
    *out = nullptr;
    if (max_jobs < 1 || slots < 1) return DEM_EINVAL;
    if (arena && ((uintptr_t)arena % ARENA_ALIGN != 0 || arena_bytes == 0)) return DEM_EINVAL;
    if (flags & ~(DEM_FLAG_NO_FORCE_OUTPUT | DEM_FLAG_RADIX_SORT | DEM_FLAG_FUSED |
                  DEM_FLAG_ACTION_REACTION | DEM_FLAG_THREAD_SPLIT | DEM_FLAG_FULL_DETECT))
        return DEM_EINVAL;
    {
        // at most one force-path variant
        const uint32_t v = flags & (DEM_FLAG_FUSED | DEM_FLAG_ACTION_REACTION | DEM_FLAG_THREAD_SPLIT);
        if (v & (v - 1)) return DEM_EINVAL;
    }
    const uint64_t mt = std::max<uint64_t>(1, tiles_of(max_particles));
    if (mt * TILE > MAX_ENTRIES || mt * TILE * slots > MAX_ENTRIES) return DEM_EINVAL;
    dem_pool* s = new (std::nothrow) dem_pool();
    if (!s) return DEM_ENOMEM;
    s->stream = (hipStream_t)stream;
    s->arena = (char*)arena;
    s->arena_bytes = arena ? arena_bytes : 0;
    s->fp64 = fp64;
    s->flags = flags;
    s->slots = slots;
    s->max_tiles = (uint32_t)mt;
    s->max_cells = std::max<uint64_t>(max_cells, 1);
    s->max_jobs = max_jobs;
    s->jobs.resize(max_jobs);
    s->segs.push_back({0, s->max_tiles, -1});
    s->free_cells.push_back({0, s->max_cells});
    const size_t np = (size_t)mt * TILE;
    dem_status r = DEM_OK;
    void *xa, *va, *ma, *xfa, *xfb, *xb, *vb, *mb;
#define ALLOC_OR_FAIL(call)   \
    do {                      \
        r = (call);           \
        if (r != DEM_OK) {    \
            destroy_pool(s);  \
            return r;         \
        }                     \
    } while (0)
    ALLOC_OR_FAIL(dalloc(s, np * sizeof(double4), &xa));
    ALLOC_OR_FAIL(dalloc(s, 3 * np * sizeof(double2), &va));
    ALLOC_OR_FAIL(dalloc(s, np, &ma));
    ALLOC_OR_FAIL(dalloc(s, np * sizeof(float4), &xfa));
    ALLOC_OR_FAIL(dalloc(s, np * sizeof(float4), &xfb));
    ALLOC_OR_FAIL(dalloc(s, np * sizeof(double4), &xb));
    ALLOC_OR_FAIL(dalloc(s, 3 * np * sizeof(double2), &vb));
    ALLOC_OR_FAIL(dalloc(s, np, &mb));
    s->S[0].xr = (double4*)xa;
    s->S[0].vw = (double2*)va;
    s->S[0].mat = (uint8_t*)ma;
    s->S[1].xr = (double4*)xb;
    s->S[1].vw = (double2*)vb;
    s->S[1].mat = (uint8_t*)mb;
    s->srt[0].xf = (float4*)xfa;
    s->srt[1].xf = (float4*)xfb;
    ALLOC_OR_FAIL(dalloc_t(s, s->max_cells, &s->cells));
    ALLOC_OR_FAIL(dalloc_t(s, np, &s->rows[0]));
    ALLOC_OR_FAIL(dalloc_t(s, np, &s->rows[1]));
    ALLOC_OR_FAIL(dalloc_t(s, np, &s->prev[0]));
    ALLOC_OR_FAIL(dalloc_t(s, np, &s->prev[1]));
    for (int k = 0; k < 2; ++k) {
        s->srt[k].xr = s->S[k].xr;
        s->srt[k].perm = s->prev[k];
    }
    ALLOC_OR_FAIL(dalloc_t(s, np, &s->keys));
    ALLOC_OR_FAIL(dalloc_t(s, np, &s->vals));
    ALLOC_OR_FAIL(dalloc_t(s, np, &s->keys_t));
    ALLOC_OR_FAIL(dalloc_t(s, np, &s->vals_t));
    ALLOC_OR_FAIL(dalloc_t(s, sort_hist_words((uint32_t)np), &s->tile_hist));
    ALLOC_OR_FAIL(dalloc_t(s, 256, &s->digit_tot));
    ALLOC_OR_FAIL(dalloc_t(s, np, &s->oldkeys));
    ALLOC_OR_FAIL(dalloc_t(s, MAX_MOVERS, &s->movers));
    ALLOC_OR_FAIL(dalloc_t(s, MAX_MOVERS, &s->mk));
    ALLOC_OR_FAIL(dalloc_t(s, MAX_MOVERS, &s->mp));
    ALLOC_OR_FAIL(dalloc(s, 6 * np * (fp64 ? 8 : 4), &s->fo));
    ALLOC_OR_FAIL(dalloc_t(s, max_jobs, &s->mats));
    ALLOC_OR_FAIL(dalloc_t(s, max_jobs, &s->jobs_d[0]));
    ALLOC_OR_FAIL(dalloc_t(s, max_jobs, &s->jobs_d[1]));
    ALLOC_OR_FAIL(dalloc_t(s, (size_t)max_jobs * DEM_MAX_WALLS, &s->walls_d));
    ALLOC_OR_FAIL(dalloc_t(s, max_jobs, &s->job_fail));
    ALLOC_OR_FAIL(dalloc_t(s, mt, &s->tile_job));
    ALLOC_OR_FAIL(dalloc_t(s, mt, &s->tile_key));
    ALLOC_OR_FAIL(dalloc_t(s, mt, &s->ts));
    ALLOC_OR_FAIL(dalloc_t(s, 1, &s->st));
    ALLOC_OR_FAIL(alloc_contacts(s, slots, &s->col_j, &s->tab_pid[0], &s->tab_pid[1],
                                 &s->tab_dt[0], &s->tab_dt[1]));
    if (flags & DEM_FLAG_ACTION_REACTION)
        ALLOC_OR_FAIL(dalloc(s, 6 * mt * TILE * slots * (fp64 ? 8 : 4), &s->pf));
    if (half_search(flags)) {
        ALLOC_OR_FAIL(dalloc_t(s, np, &s->deg));
        ALLOC_OR_FAIL(dalloc_t(s, np * 8, &s->adj));
        s->adj_slots = 8;
    }
#undef ALLOC_OR_FAIL
    s->cap = (uint64_t)mt * TILE * slots;
    hipError_t e = hipMemset(s->st, 0, sizeof(Status));
    if (e == hipSuccess) e = hipMemset(s->ts, 0, mt * sizeof(TileStats));
    if (e == hipSuccess) e = hipMemset(s->cells, 0, s->max_cells * sizeof(uint2));
    if (e == hipSuccess) e = hipMemset(s->rows[0], 0, np * sizeof(uint2));
    if (e == hipSuccess) e = hipMemset(s->rows[1], 0, np * sizeof(uint2));
    if (e == hipSuccess) e = hipMemset(s->fo, 0, 6 * np * (fp64 ? 8 : 4));
    if (e == hipSuccess && s->deg) e = hipMemset(s->deg, 0, np * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMemset(s->jobs_d[0], 0, max_jobs * sizeof(Job));
    if (e == hipSuccess) e = hipMemset(s->jobs_d[1], 0, max_jobs * sizeof(Job));
    if (e == hipSuccess) e = hipMemset(s->job_fail, 0, max_jobs * sizeof(uint32_t));
    if (e == hipSuccess) e = hipMemset(s->S[0].mat, 0, np);
    if (e == hipSuccess) e = hipMemset(s->S[1].mat, 0, np);
    std::vector<uint32_t> tj(mt, NO_JOB);
    if (e == hipSuccess) e = hipMemcpy(s->tile_job, tj.data(), mt * 4, hipMemcpyHostToDevice);
    {
        // every permutation entry starts as the identity (ghost slots and
        // free tiles keep theirs; the kernels also clamp what they read)
        std::vector<uint32_t> id(np);
        std::iota(id.begin(), id.end(), 0u);
        for (int k = 0; k < 2 && e == hipSuccess; ++k)
            e = hipMemcpy(s->prev[k], id.data(), np * 4, hipMemcpyHostToDevice);
    }
    if (e == hipSuccess) e = hipMemset(s->tile_key, 0, mt * 4);
    if (e != hipSuccess) {
        destroy_pool(s);
        return hip_status(e);
    }
    *out = s;
    return DEM_OK;
}

int seg_bits(size_t nsegs) {
    int jb = 0;
    while ((size_t(1) << jb) < nsegs) ++jb;
    return jb;
}

// Ranks of the segments in memory order are the high bits of the sort key,
// so one sort keeps every job (and every free gap) inside its segment.
dem_status upload_layout(dem_pool* s) {
    int lb = 1;
    bool per = false, mm = false;
    for (const HostJob& j : s->jobs)
        if (j.used) {
            lb = std::max(lb, j.lay.key_bits);
            per = per || j.P.periodic != 0;
            mm = mm || j.multi_mat;
        }
    const int jb = seg_bits(s->segs.size());
    if (lb + jb > 32) return DEM_EBUSY;
    s->lb = lb;
    s->any_periodic = per;
    s->any_multi_mat = mm;
    std::vector<uint32_t> tj(s->max_tiles, NO_JOB), tk(s->max_tiles, 0u);
    uint32_t hw = 0;
    for (size_t q = 0; q < s->segs.size(); ++q) {
        const Seg& g = s->segs[q];
        const uint32_t key = lb >= 32 ? 0u : (uint32_t)((uint64_t)q << lb);
        for (uint32_t t = g.start; t < g.start + g.len; ++t) {
            tj[t] = g.slot < 0 ? NO_JOB : (uint32_t)g.slot;
            tk[t] = key;
        }
        if (g.slot >= 0) hw = std::max(hw, g.start + g.len);
    }
    s->hw_tiles = hw;
    dem_status r = upload(s, s->tile_job, tj.data(), s->max_tiles * 4);
    if (r == DEM_OK) r = upload(s, s->tile_key, tk.data(), s->max_tiles * 4);
    return r;
}

int take_tiles(dem_pool* s, uint32_t need, int slot) {
    for (size_t q = 0; q < s->segs.size(); ++q) {
        Seg& g = s->segs[q];
        if (g.slot >= 0 || g.len < need) continue;
        const uint32_t start = g.start;
        if (g.len == need) {
            g.slot = slot;
        } else {
            Seg rest{start + need, g.len - need, -1};
            g.len = need;
            g.slot = slot;
            s->segs.insert(s->segs.begin() + q + 1, rest);
        }
        return (int)start;
    }
    return -1;
}

void release_tiles(dem_pool* s, int slot) {
    for (Seg& g : s->segs)
        if (g.slot == slot) g.slot = -1;
    std::vector<Seg> m;
    for (const Seg& g : s->segs) {
        if (g.len == 0 && g.slot < 0) continue;
        if (!m.empty() && m.back().slot < 0 && g.slot < 0) m.back().len += g.len;
        else m.push_back(g);
    }
    if (m.empty()) m.push_back({0, s->max_tiles, -1});
    s->segs = m;
}

long long take_cells(dem_pool* s, uint64_t need) {
    for (auto& f : s->free_cells)
        if (f.second >= need) {
            const uint64_t start = f.first;
            f.first += need;
            f.second -= need;
            return (long long)start;
        }
    return -1;
}

void release_cells(dem_pool* s, uint64_t start, uint64_t len) {
    s->free_cells.push_back({start, len});
    std::sort(s->free_cells.begin(), s->free_cells.end());
    std::vector<std::pair<uint64_t, uint64_t>> m;
    for (auto& f : s->free_cells) {
        if (!f.second) continue;
        if (!m.empty() && m.back().first + m.back().second == f.first) m.back().second += f.second;
        else m.push_back(f);
    }
    s->free_cells = m;
}

// Host-side placement of a job's particles in cell order (stable by particle
// id) with its cell bounds relative to the job's first position: the device
// only ever re-sorts jobs it already has.
struct Placed {
    std::vector<double4> xr;
    std::vector<float4> xf;
    std::vector<double2> vw0, vw1, vw2;
    std::vector<uint8_t> mat;
    std::vector<uint2> cells;  // (start, end) relative to the job; (0, 0) = empty
};

uint32_t host_cell_coord(const Geo& G, double x, int a) {
    double f = std::floor((x - G.lo[a]) * G.inv_cell[a]);
    if (!(f >= 0.0)) return 0;
    if (f >= (double)G.nc[a]) return (uint32_t)G.nc[a] - 1;
    return (uint32_t)f;
}

void place_job(const HostJob& J, const double* x, const double* v, const double* w, Placed& out) {
    const uint64_t n = J.n;
    const Geo& G = J.geo;
    std::vector<uint32_t> key(n), lin(n);
    for (uint64_t i = 0; i < n; ++i) {
        const uint32_t cx = host_cell_coord(G, x[3 * i], 0), cy = host_cell_coord(G, x[3 * i + 1], 1),
                       cz = host_cell_coord(G, x[3 * i + 2], 2);
        key[i] = ((spread2_host(cy) | (spread2_host(cz) << 1)) << G.xbits) | cx;
        lin[i] = (cz * (uint32_t)G.nc[1] + cy) * (uint32_t)G.nc[0] + cx;
    }
    std::vector<uint32_t> order(n);
    std::iota(order.begin(), order.end(), 0u);
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) { return key[a] < key[b]; });
    out.xr.resize(n);
    out.xf.resize(n);
    out.vw0.resize(n);
    out.vw1.resize(n);
    out.vw2.resize(n);
    out.mat.resize(n);
    out.cells.assign(J.ncells, make_uint2(0, 0));
    const float qnan = std::nanf("");
    for (uint64_t q = 0; q < n; ++q) {
        const uint32_t i = order[q];
        uint64_t meta = pack_meta(J.r[i], i);
        double mw;
        std::memcpy(&mw, &meta, 8);
        out.xr[q] = make_double4(x[3 * i], x[3 * i + 1], x[3 * i + 2], mw);
        const double rx = x[3 * i] - G.lo[0], ry = x[3 * i + 1] - G.lo[1], rz = x[3 * i + 2] - G.lo[2];
        const bool near = std::fabs(rx) <= 3.0 * G.L[0] && std::fabs(ry) <= 3.0 * G.L[1] &&
                          std::fabs(rz) <= 3.0 * G.L[2];
        out.xf[q] = near ? make_float4((float)rx, (float)ry, (float)rz, J.r[i])
                         : make_float4(qnan, qnan, qnan, J.r[i]);
        out.vw0[q] = make_double2(v[3 * i], v[3 * i + 1]);
        out.vw1[q] = make_double2(v[3 * i + 2], w[3 * i]);
        out.vw2[q] = make_double2(w[3 * i + 1], w[3 * i + 2]);
        out.mat[q] = (uint8_t)J.mat[i];
        const uint32_t k = key[i];
        if (q == 0 || key[order[q - 1]] != k) out.cells[lin[i]].x = (uint32_t)q;
        if (q + 1 == n || key[order[q + 1]] != k) out.cells[lin[i]].y = (uint32_t)q + 1;
    }
}

// Upload a placed job (its state, cells, an empty history and identity map,
// its descriptor and materials) at its tiles and cells.
dem_status upload_job(dem_pool* s, int slot, Placed& pl, double t0, uint32_t steps) {
    HostJob& J = s->jobs[slot];
    const uint32_t p0 = J.tile0 * TILE;
    for (uint2& c : pl.cells)
        if (c.y > c.x) {
            c.x += p0;
            c.y += p0;
        }
    const uint64_t n = J.n, np = (uint64_t)s->max_tiles * TILE;
    dem_status r = DEM_OK;
    auto up = [&](void* dst, const void* src, size_t bytes) {
        if (r == DEM_OK) r = upload(s, dst, src, bytes);
    };
    auto upv = [&](void* dst, auto& v) {
        if (r == DEM_OK) r = upload_vec(s, dst, v);
    };
    // the state into the current buffer, in sorted order (its permutation
    // is the identity)
    State& X = s->S[s->cur];
    upv(X.xr + p0, pl.xr);
    upv(s->srt[s->cur].xf + p0, pl.xf);
    upv(X.vw + p0, pl.vw0);
    upv(X.vw + np + p0, pl.vw1);
    upv(X.vw + 2 * np + p0, pl.vw2);
    upv(X.mat + p0, pl.mat);
    upv(s->cells + J.cell_base, pl.cells);
    const uint64_t span = (uint64_t)J.ntiles * TILE;
    std::vector<uint2> zr(span, make_uint2(0, 0));
    std::vector<uint32_t> idp(span);
    std::iota(idp.begin(), idp.end(), p0);
    up(s->rows[s->cur] + p0, zr.data(), span * sizeof(uint2));
    up(s->prev[s->cur] + p0, idp.data(), span * 4);
    std::vector<TileStats> z(J.ntiles);
    if (J.ntiles) std::memset(z.data(), 0, z.size() * sizeof(TileStats));
    up(s->ts + J.tile0, z.data(), J.ntiles * sizeof(TileStats));
    // F, T of a new job read as zero until its first step
    const size_t fs = s->fp64 ? 8 : 4;
    if (span) {
        std::vector<char> zf(span * fs, 0);
        for (int c = 0; c < 6; ++c) up((char*)s->fo + ((size_t)c * np + p0) * fs, zf.data(), span * fs);
    }
    MatTable mt;
    fill_mat_table(J.P, J.mats, mt);
    up(s->mats + slot, &mt, sizeof(MatTable));
    Job jd;
    std::memset(&jd, 0, sizeof(jd));
    jd.g = J.geo;
    jd.g.le_shift = le_offset(J.geo, t0);
    jd.g.le_shift_next = le_offset(J.geo, t0 + J.geo.dt);
    jd.t = t0;
    jd.margin = detect_margin(J.geo);
    jd.p0 = p0;
    jd.n = (uint32_t)n;
    jd.cell_base = J.cell_base;
    jd.mat = (uint32_t)slot;
    jd.status = JOB_ACTIVE;
    jd.steps_left = steps;
    jd.nxw = (uint32_t)J.walls.size();
    jd.xw = s->walls_d + (size_t)slot * DEM_MAX_WALLS;
    if (!J.walls.empty()) up(s->walls_d + (size_t)slot * DEM_MAX_WALLS, J.walls.data(),
                             J.walls.size() * sizeof(dem_wall));
    up(s->jobs_d[s->cur] + slot, &jd, sizeof(Job));
    const uint32_t zero = 0;
    up(s->job_fail + slot, &zero, sizeof(zero));
    return r;
}

// A job before it has a place in a pool: validated constants, grid, time
// step and its particles in cell order.  Host work only.
struct Prepared {
    HostJob J;
    Placed pl;
};

dem_status prepare_job(const dem_params* params, const dem_material* mats, uint32_t n_mats,
                       uint64_t n, const double* x, const double* v, const double* w,
                       const float* radius, const uint16_t* mat_id, bool two_level,
                       Prepared& pj) {
    dem_status r = validate(params, mats, n_mats);
    if (r != DEM_OK) return r;
    if (n >= (uint64_t)FACE) return DEM_EINVAL;
    if (n && (!x || !v || !w || !radius)) return DEM_EINVAL;
    double rmax = 0.0;
    for (uint64_t i = 0; i < n; ++i) {
        if (!(radius[i] > 0.0f) || !std::isfinite(radius[i])) return DEM_EINVAL;
        if (!finite3(x + 3 * i) || !finite3(v + 3 * i) || !finite3(w + 3 * i)) return DEM_EINVAL;
        if (!in_periodic_box(*params, x + 3 * i)) return DEM_EINVAL;
        if (mat_id && mat_id[i] >= n_mats) return DEM_EINVAL;
        rmax = std::max(rmax, (double)radius[i]);
    }
    if (n == 0) {
        double lmin = INFINITY;
        for (int a = 0; a < 3; ++a) lmin = std::min(lmin, params->hi[a] - params->lo[a]);
        rmax = lmin / 6.1;
    }
    Layout lay;
    double used = rmax;
    r = plan_job_grid(*params, rmax, two_level ? radius_cut(*params, radius, n, rmax) : rmax, n,
                      lay, used);
    if (r != DEM_OK) return r;
    HostJob& J = pj.J;
    J = HostJob();
    J.two_level = two_level;
    J.P = *params;
    J.walls.assign(params->extra_walls, params->extra_walls + params->n_extra_walls);
    J.P.extra_walls = nullptr;
    J.mats.assign(mats, mats + n_mats);
    J.n = n;
    J.ntiles = (uint32_t)tiles_of(n);
    J.ncells = (uint32_t)((uint64_t)lay.nc[0] * lay.nc[1] * lay.nc[2]);
    J.lay = lay;
    J.multi_mat = n_mats > 1;
    J.r.assign(radius, radius + n);
    J.mat.assign(n, 0);
    if (mat_id) J.mat.assign(mat_id, mat_id + n);
    Geo& G = J.geo;
    std::memset(&G, 0, sizeof(G));
    for (int a = 0; a < 3; ++a) {
        G.lo[a] = params->lo[a];
        G.hi[a] = params->hi[a];
        G.L[a] = params->hi[a] - params->lo[a];
        G.inv_cell[a] = 1.0 / lay.cell[a];
        G.cw[a] = lay.cell[a];
        G.inv_L[a] = 1.0 / G.L[a];
        G.nc[a] = lay.nc[a];
        G.g[a] = params->gravity[a];
    }
    // the cell of a coordinate is computed in floating point, so a partner
    // may sit a few rounding units outside its cell's slab
    double span = 0.0;
    for (int a = 0; a < 3; ++a) span = std::max(span, std::fabs(G.lo[a]) + std::fabs(G.hi[a]));
    set_cut(G, used, rmax, span);
    G.walls = params->walls;
    G.periodic = params->periodic;
    G.le = params->shear_rate != 0.0;
    G.key_bits = lay.key_bits;
    G.xbits = lay.xbits;
    G.le_dv = params->shear_rate * G.L[1];
    // time step: t_c / 50 of two spheres of the smallest radius at 0.1 m/s
    double dt = params->dt;
    if (dt == 0.0) {
        if (n == 0) {
            dt = 1e-9;
        } else {
            uint64_t k = 0;
            for (uint64_t i = 1; i < n; ++i)
                if (radius[i] < radius[k]) k = i;
            const int m = mat_id ? mat_id[k] : 0;
            MatTable mt;
            fill_mat_table(*params, J.mats, mt);
            const double rk = (double)radius[k];
            const double mk = mt.mass_pref[m] * rk * rk * rk;
            const double kn = mt.kn_pref[m * MAXMAT + m] * std::sqrt(rk * rk / (rk + rk));
            dt = hertz_contact_time(0.5 * mk, kn, 0.1) / 50.0;
        }
    }
    G.dt = dt;
    place_job(J, x, v, w, pj.pl);
    return DEM_OK;
}

// Give a prepared job a slot, tiles and cells in the pool and upload it.
// The pool must have no unconfirmed steps.
dem_status commit_job(dem_pool* s, Prepared& pj, uint32_t steps, int* slot_out) {
    const HostJob& P = pj.J;
    if ((P.P.precision == DEM_PREC_FP64) != s->fp64) return DEM_EINVAL;
    if (P.n > (uint64_t)s->max_tiles * TILE) return DEM_EBUSY;
    int slot = -1;
    for (uint32_t k = 0; k < s->max_jobs; ++k)
        if (!s->jobs[k].used) {
            slot = (int)k;
            break;
        }
    if (slot < 0) return DEM_EBUSY;
    const long long cb = take_cells(s, P.ncells);
    if (cb < 0) return DEM_EBUSY;
    const int t0 = take_tiles(s, P.ntiles, slot);
    if (t0 < 0) {
        release_cells(s, (uint64_t)cb, P.ncells);
        return DEM_EBUSY;
    }
    HostJob& J = s->jobs[slot];
    J = std::move(pj.J);
    J.used = true;
    J.id = s->next_id++;
    J.tile0 = (uint32_t)t0;
    J.cell_base = (uint32_t)cb;
    dem_status r = upload_layout(s);
    if (r == DEM_OK) r = upload_job(s, slot, pj.pl, J.P.time, steps);
    if (r != DEM_OK) {
        release_tiles(s, slot);
        release_cells(s, J.cell_base, J.ncells);
        J = HostJob();
        (void)upload_layout(s);
        return r;
    }
    *slot_out = slot;
    return DEM_OK;
}

dem_status remove_job(dem_pool* s, int slot) {
    HostJob& J = s->jobs[slot];
    if (!J.used) return DEM_EINVAL;
    release_tiles(s, slot);
    release_cells(s, J.cell_base, J.ncells);
    J = HostJob();
    return upload_layout(s);
}

// ------------------------------------------------------------ step pipeline
PoolView view(dem_pool* s) {
    PoolView P;
    P.jobs = s->jobs_d[s->cur];
    P.job_fail = s->job_fail;
    P.tile_job = s->tile_job;
    P.tile_key = s->tile_key;
    P.ntiles = s->hw_tiles;
    P.ns = s->max_tiles * TILE;
    P.lmask = s->lb >= 32 ? 0xFFFFFFFFu : ((1u << s->lb) - 1u);
    P.mats = s->mats;
    P.ts = s->ts;
    P.st = s->st;
    P.any_periodic = s->any_periodic;
    return P;
}

void prof_record(dem_pool* s, size_t slot, int ev) {
    if (!s->prof) return;
    (void)hipEventRecord(s->prof_ev[slot].e[ev], s->stream);
}

// One step of every running job; `o` is the buffer holding the old table.
dem_status enqueue_step(dem_pool* s, int o) {
    const int w = 1 - o;
    PoolView P = view(s);
    P.jobs = s->jobs_d[o];
    // the step reads the state and job descriptors of buffer o and writes
    // those of buffer w
    State X = s->S[o], Y = s->S[w];
    if (!s->any_multi_mat) X.mat = Y.mat = nullptr;
    size_t slot = 0;
    if (s->prof) {
        if (s->prof_used == s->prof_ev.size()) {
            ProfEv pe;
            for (int q = 0; q <= DEM_NPHASE; ++q) HIPCHK(hipEventCreate(&pe.e[q]));
            s->prof_ev.push_back(pe);
        }
        slot = s->prof_used++;
    }
    // the fused single loop replaces detect and force (the detect phase is
    // then empty)
    const bool fused = (s->flags & DEM_FLAG_FUSED) != 0;
    prof_record(s, slot, 0);
    const bool half = half_search(s->flags);
    if (half)
        launch_detect_half(P, s->kmax, s->srt[o], s->cells, s->deg, s->adj, s->stream);
    else if (!fused)
        launch_detect(P, s->kmax, s->srt[o], s->cells, s->rows[w], s->col_j, s->slots, s->stream);
    prof_record(s, slot, 1);
    // the merge sort unless a recent step had too many cell changes
    const bool merge = s->radix_left == 0 && !(s->flags & DEM_FLAG_RADIX_SORT);
    if (s->radix_left) s->radix_left--;
    void* fo = (s->flags & DEM_FLAG_NO_FORCE_OUTPUT) ? nullptr : s->fo;
    if (s->flags & DEM_FLAG_ACTION_REACTION)
        launch_action_reaction(P, s->fp64, s->srt[o], X, Y, s->rows[w], s->col_j, s->rows[o],
                               s->prev[o], s->tab_pid[o], s->tab_dt[o], s->tab_pid[w], s->tab_dt[w],
                               s->cap, s->pf, s->cells, s->keys, s->vals, fo,
                               merge ? s->oldkeys : nullptr, merge ? s->movers : nullptr,
                               s->stream);
    else if (s->flags & DEM_FLAG_THREAD_SPLIT)
        launch_force_thread(P, s->fp64, s->srt[o], X, Y, s->rows[w], s->col_j, s->rows[o], s->prev[o],
                            s->tab_pid[o], s->tab_dt[o], s->tab_pid[w], s->tab_dt[w], s->cap,
                            s->cells, s->keys, s->vals, fo, merge ? s->oldkeys : nullptr,
                            merge ? s->movers : nullptr, s->stream);
    else if (fused)
        launch_fused(P, s->fp64, s->srt[o], X, Y, s->rows[w], s->col_j, s->rows[o], s->prev[o],
                     s->tab_pid[o], s->tab_dt[o], s->tab_pid[w], s->tab_dt[w], s->cap, s->slots,
                     s->cells, s->keys, s->vals, fo, merge ? s->oldkeys : nullptr,
                     merge ? s->movers : nullptr, s->stream);
    else if (half)
        launch_force_half(P, s->fp64, s->kmax, s->srt[o], X, Y, s->deg, s->adj, s->rows[w], s->col_j,
                          s->slots, s->rows[o], s->prev[o], s->tab_pid[o], s->tab_dt[o],
                          s->tab_pid[w], s->tab_dt[w], s->cap, s->cells, s->keys, s->vals, fo,
                          merge ? s->oldkeys : nullptr, merge ? s->movers : nullptr, s->stream);
    else
        launch_force(P, s->fp64, s->srt[o], X, Y, s->rows[w], s->col_j, s->rows[o], s->prev[o],
                     s->tab_pid[o], s->tab_dt[o], s->tab_pid[w], s->tab_dt[w], s->cap, s->cells,
                     s->keys, s->vals, fo, merge ? s->oldkeys : nullptr,
                     merge ? s->movers : nullptr, s->stream);
    prof_record(s, slot, 2);
    uint32_t *ko, *vo;
    if (merge) {
        launch_merge_sort(P, s->oldkeys, s->movers, s->mk, s->mp, s->keys_t, Y, s->srt[w],
                          s->prev[w], s->cells, s->jobs_d[w], s->max_jobs, s->stream);
        ko = s->keys_t;
        vo = s->vals_t;
    } else {
        launch_radix_sort(s->keys, s->vals, s->keys_t, s->vals_t, s->hw_tiles * TILE,
                          s->lb + seg_bits(s->segs.size()), s->tile_hist, s->digit_tot, &ko, &vo,
                          s->st, s->stream);
    }
    prof_record(s, slot, 3);
    launch_reorder(P, s->jobs_d[w], s->max_jobs, !merge, ko, vo, Y, s->srt[w], s->prev[w], s->cells,
                   s->stream);
    prof_record(s, slot, 4);
    HIPCHK(hipGetLastError());
    return DEM_OK;
}

dem_status step_impl(dem_pool* s, uint32_t nsteps) {
    if (s->failed != DEM_OK) return s->failed;
    for (uint32_t q = 0; q < nsteps; ++q) {
        dem_status r = enqueue_step(s, s->cur);
        if (r != DEM_OK) return r;
        s->pending.push_back(s->cur);
        s->cur = 1 - s->cur;
    }
    return DEM_OK;
}

dem_status read_status(dem_pool* s, Status& h) {
    HIPCHK(hipStreamSynchronize(s->stream));
    HIPCHK(hipMemcpy(&h, s->st, sizeof(Status), hipMemcpyDeviceToHost));
    return DEM_OK;
}

// Grow every tile's region of the contact table to hold `need` contacts per
// tile, keeping the old table of buffer `o` at the same positions (its rows
// hold absolute indices).
dem_status regrow(dem_pool* s, uint64_t need_per_tile, int o) {
    const uint64_t nt = s->max_tiles;
    uint64_t ns = std::max<uint64_t>((uint64_t)s->slots * 2, (need_per_tile + TILE - 1) / TILE + 2);
    if (nt * TILE * ns > MAX_ENTRIES) ns = MAX_ENTRIES / (nt * TILE);
    if (ns <= s->slots) return DEM_ECAPACITY;
    const uint64_t oc = s->cap;
    uint32_t *col, *p0, *p1;
    double *d0, *d1;
    if (alloc_contacts(s, (uint32_t)ns, &col, &p0, &p1, &d0, &d1) != DEM_OK) return DEM_ECAPACITY;
    void* pf = nullptr;
    if (s->flags & DEM_FLAG_ACTION_REACTION) {
        if (dalloc(s, 6 * nt * TILE * ns * (s->fp64 ? 8 : 4), &pf) != DEM_OK) {
            dfree(s, col);
            dfree(s, p0);
            dfree(s, p1);
            dfree(s, d0);
            dfree(s, d1);
            return DEM_ECAPACITY;
        }
    }
    const uint64_t nc = nt * TILE * ns;
    uint32_t* np_[2] = {p0, p1};
    double* nd_[2] = {d0, d1};
    HIPCHK(hipMemcpyAsync(np_[o], s->tab_pid[o], oc * 4, hipMemcpyDeviceToDevice, s->stream));
    for (int c = 0; c < 3; ++c)
        HIPCHK(hipMemcpyAsync(nd_[o] + (size_t)c * nc, s->tab_dt[o] + (size_t)c * oc, oc * 8,
                              hipMemcpyDeviceToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    dfree(s, s->col_j);
    for (int k = 0; k < 2; ++k) {
        dfree(s, s->tab_pid[k]);
        dfree(s, s->tab_dt[k]);
    }
    if (pf) {
        dfree(s, s->pf);
        s->pf = pf;
    }
    s->col_j = col;
    s->tab_pid[0] = p0;
    s->tab_pid[1] = p1;
    s->tab_dt[0] = d0;
    s->tab_dt[1] = d1;
    s->cap = nc;
    s->slots = (uint32_t)ns;
    s->regrows++;
    return DEM_OK;
}

dem_status sync_impl(dem_pool* s) {
    if (s->failed != DEM_OK) return s->failed;
    for (;;) {
        Status h;
        dem_status r = read_status(s, h);
        if (r != DEM_OK) return r;
        s->staging.clear();
        s->held.clear();
        while (s->steps_confirmed < h.steps_done && !s->pending.empty()) {
            s->pending.pop_front();
            s->steps_confirmed++;
        }
        if (h.err == 0) return DEM_OK;
        // a step failed pool-wide before changing any state: fix and redo
        const int o = s->pending.empty() ? s->cur : s->pending.front();
        if (h.err & ERR_ROW) {
            if (s->kmax >= 32) {
                s->failed = DEM_ECAPACITY;
                return DEM_ECAPACITY;
            }
            s->kmax = s->kmax <= 8 ? 16 : 32;
            if (s->adj && s->adj_slots < s->kmax) {
                // longer adjacency lists for the half search (their contents
                // live within one step)
                uint2* a2 = nullptr;
                r = dalloc_t(s, (size_t)s->max_tiles * TILE * s->kmax, &a2);
                if (r != DEM_OK) {
                    // a lent arena without room left is a capacity limit
                    s->failed = s->arena ? DEM_ECAPACITY : r;
                    return s->failed;
                }
                dfree(s, s->adj);
                s->adj = a2;
                s->adj_slots = s->kmax;
            }
        }
        if (h.err & ERR_MOVERS) s->radix_left = 16 + (uint32_t)s->pending.size();
        if (h.err & ERR_CAPACITY) {
            r = regrow(s, h.need, o);
            if (r != DEM_OK) {
                s->failed = r;
                return r;
            }
        }
        Status z = h;
        z.err = 0;
        z.need = 0;
        z.movers = 0;
        HIPCHK(hipMemcpy(s->st, &z, sizeof(Status), hipMemcpyHostToDevice));
        // the abandoned step may have emptied cell bounds (the force kernel
        // does so as it runs): restore those of the order it started from
        PoolView Pv = view(s);
        Pv.jobs = s->jobs_d[o];
        launch_rebuild_cells(Pv, s->srt[o], s->cells, s->stream);
        HIPCHK(hipGetLastError());
        s->prof_used = 0;
        const size_t k = s->pending.size();
        s->pending.clear();
        s->cur = o;
        r = step_impl(s, (uint32_t)k);
        if (r != DEM_OK) return r;
    }
}

dem_status read_job(dem_pool* s, int slot, Job& jd) {
    HIPCHK(hipMemcpy(&jd, s->jobs_d[s->cur] + slot, sizeof(Job), hipMemcpyDeviceToHost));
    return DEM_OK;
}

// pids of a job's positions in the current state buffer: the order in which
// the last step wrote its state, forces and contact rows
dem_status job_pids(dem_pool* s, const HostJob& J, std::vector<uint32_t>& pid) {
    const uint64_t n = J.n;
    std::vector<double4> xr(n);
    pid.resize(n);
    const uint32_t p0 = J.tile0 * TILE;
    if (n) HIPCHK(hipMemcpy(xr.data(), s->S[s->cur].xr + p0, n * sizeof(double4),
                            hipMemcpyDeviceToHost));
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t m;
        std::memcpy(&m, &xr[i].w, 8);
        pid[i] = (uint32_t)(m >> 32);
    }
    return DEM_OK;
}

dem_status get_state_impl(dem_pool* s, int slot, double* x, double* v, double* w, double* F,
                          double* T) {
    const HostJob& J = s->jobs[slot];
    const uint64_t n = J.n, np = (uint64_t)s->max_tiles * TILE;
    const uint32_t p0 = J.tile0 * TILE;
    if (n == 0) return DEM_OK;
    std::vector<double4> xr(n);
    std::vector<double2> v0(n), v1(n), v2(n);
    const State& X = s->S[s->cur];
    HIPCHK(hipMemcpy(xr.data(), X.xr + p0, n * sizeof(double4), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(v0.data(), X.vw + p0, n * sizeof(double2), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(v1.data(), X.vw + np + p0, n * sizeof(double2), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(v2.data(), X.vw + 2 * np + p0, n * sizeof(double2), hipMemcpyDeviceToHost));
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t m;
        std::memcpy(&m, &xr[i].w, 8);
        const uint32_t p = (uint32_t)(m >> 32);
        if (x) {
            x[3 * p] = xr[i].x;
            x[3 * p + 1] = xr[i].y;
            x[3 * p + 2] = xr[i].z;
        }
        if (v) {
            v[3 * p] = v0[i].x;
            v[3 * p + 1] = v0[i].y;
            v[3 * p + 2] = v1[i].x;
        }
        if (w) {
            w[3 * p] = v1[i].y;
            w[3 * p + 1] = v2[i].x;
            w[3 * p + 2] = v2[i].y;
        }
    }
    if (F || T) {
        // F, T were written at the positions of the current buffer (zero
        // before the first step)
        std::vector<uint32_t> pid;
        dem_status r = job_pids(s, J, pid);
        if (r != DEM_OK) return r;
        std::vector<double> f(6 * n);
        for (int c = 0; c < 6; ++c) {
            if (s->fp64) {
                HIPCHK(hipMemcpy(f.data() + c * n, (double*)s->fo + (size_t)c * np + p0, n * 8,
                                 hipMemcpyDeviceToHost));
            } else {
                std::vector<float> ff(n);
                HIPCHK(hipMemcpy(ff.data(), (float*)s->fo + (size_t)c * np + p0, n * 4,
                                 hipMemcpyDeviceToHost));
                for (uint64_t k = 0; k < n; ++k) f[c * n + k] = ff[k];
            }
        }
        for (uint64_t i = 0; i < n; ++i) {
            const uint32_t p = pid[i];
            for (int a = 0; a < 3; ++a) {
                if (F) F[3 * p + a] = f[a * n + i];
                if (T) T[3 * p + a] = f[(3 + a) * n + i];
            }
        }
    }
    return DEM_OK;
}

struct Contact {
    uint32_t i, j;
    double dt[3];
};

dem_status read_contacts(dem_pool* s, int slot, std::vector<Contact>& out) {
    out.clear();
    const HostJob& J = s->jobs[slot];
    const uint64_t n = J.n;
    if (n == 0) return DEM_OK;
    const uint32_t p0 = J.tile0 * TILE;
    const int o = s->cur;
    std::vector<uint2> rows(n);
    HIPCHK(hipMemcpy(rows.data(), s->rows[o] + p0, n * sizeof(uint2), hipMemcpyDeviceToHost));
    uint64_t lo = ~0ull, hi = 0;
    for (const uint2& q : rows)
        if (q.y) {
            lo = std::min<uint64_t>(lo, q.x);
            hi = std::max<uint64_t>(hi, (uint64_t)q.x + q.y);
        }
    std::vector<uint32_t> pid;
    dem_status r = job_pids(s, J, pid);
    if (r != DEM_OK) return r;
    if (hi <= lo) return DEM_OK;
    const uint64_t m = hi - lo;
    std::vector<uint32_t> tp(m);
    std::vector<double> td(3 * m);
    HIPCHK(hipMemcpy(tp.data(), s->tab_pid[o] + lo, m * 4, hipMemcpyDeviceToHost));
    for (int a = 0; a < 3; ++a)
        HIPCHK(hipMemcpy(td.data() + a * m, s->tab_dt[o] + (size_t)a * s->cap + lo, m * 8,
                         hipMemcpyDeviceToHost));
    for (uint64_t p = 0; p < n; ++p)
        for (uint32_t k = rows[p].x; k < rows[p].x + rows[p].y; ++k) {
            const uint64_t q = k - lo;
            out.push_back({pid[p], tp[q], {td[q], td[m + q], td[2 * m + q]}});
        }
    std::sort(out.begin(), out.end(), [](const Contact& a, const Contact& b) {
        return a.i < b.i || (a.i == b.i && a.j < b.j);
    });
    if (s->flags & DEM_FLAG_ACTION_REACTION) {
        // a pair's displacement is kept by its owner (the lower id); the other
        // directed contact carries its negative
        for (Contact& c : out) {
            if (c.j >= FACE || c.j > c.i) continue;
            const Contact key{c.j, c.i, {0, 0, 0}};
            auto it = std::lower_bound(out.begin(), out.end(), key,
                                       [](const Contact& a, const Contact& b) {
                                           return a.i < b.i || (a.i == b.i && a.j < b.j);
                                       });
            if (it != out.end() && it->i == c.j && it->j == c.i)
                for (int a = 0; a < 3; ++a) c.dt[a] = -it->dt[a];
        }
    }
    return DEM_OK;
}

// Install a history (pid keyed) as the old table of the job's next step, at
// the positions of the current state buffer (which the next step reaches
// through its permutation), inside the job's own tile regions.
dem_status write_contacts(dem_pool* s, int slot, std::vector<Contact>& c) {
    HostJob& J = s->jobs[slot];
    const uint64_t n = J.n;
    std::sort(c.begin(), c.end(), [](const Contact& a, const Contact& b) {
        return a.i < b.i || (a.i == b.i && a.j < b.j);
    });
    for (size_t k = 0; k < c.size(); ++k) {
        if (c[k].i >= n) return DEM_EINVAL;
        if (c[k].j >= n && c[k].j < FACE) return DEM_EINVAL;
        if (c[k].j >= FACE + 6 + (uint32_t)J.walls.size()) return DEM_EINVAL;
        if (c[k].j == c[k].i) return DEM_EINVAL;
        if (k && c[k].i == c[k - 1].i && c[k].j == c[k - 1].j) return DEM_EINVAL;
        if (!finite3(c[k].dt)) return DEM_EINVAL;
    }
    const uint64_t span = (uint64_t)J.ntiles * TILE;
    while (c.size() > span * s->slots) {
        dem_status r = regrow(s, (c.size() + J.ntiles - 1) / std::max<uint32_t>(J.ntiles, 1), s->cur);
        if (r != DEM_OK) return r;
    }
    std::vector<uint32_t> pid;
    dem_status r = job_pids(s, J, pid);
    if (r != DEM_OK) return r;
    std::vector<uint32_t> pos(n);
    for (uint64_t q = 0; q < n; ++q) pos[pid[q]] = (uint32_t)q;
    const uint32_t p0 = J.tile0 * TILE;
    const uint64_t base = (uint64_t)p0 * s->slots;
    // entries grouped by sorted position, each row in partner-id order
    std::vector<size_t> idx(c.size());
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return pos[c[a].i] < pos[c[b].i]; });
    const size_t m = c.size();
    std::vector<uint2> rows(n, make_uint2(0, 0));
    std::vector<uint32_t> tp(m);
    std::vector<double> td(3 * std::max<size_t>(m, 1));
    for (size_t k = 0; k < m; ++k) {
        const Contact& e = c[idx[k]];
        uint2& rw = rows[pos[e.i]];
        if (rw.y == 0) rw.x = (uint32_t)(base + k);
        rw.y++;
        tp[k] = e.j;
        for (int a = 0; a < 3; ++a) td[a * m + k] = e.dt[a];
    }
    const int o = s->cur;
    if (n) HIPCHK(hipMemcpy(s->rows[o] + p0, rows.data(), n * sizeof(uint2), hipMemcpyHostToDevice));
    if (m) {
        HIPCHK(hipMemcpy(s->tab_pid[o] + base, tp.data(), m * 4, hipMemcpyHostToDevice));
        for (int a = 0; a < 3; ++a)
            HIPCHK(hipMemcpy(s->tab_dt[o] + (size_t)a * s->cap + base, td.data() + a * m, m * 8,
                             hipMemcpyHostToDevice));
    }
    return DEM_OK;
}

dem_status set_state_impl(dem_pool* s, int slot, const double* x, const double* v, const double* w) {
    HostJob& J = s->jobs[slot];
    for (uint64_t k = 0; k < J.n; ++k)
        if (!finite3(x + 3 * k) || !finite3(v + 3 * k) || !finite3(w + 3 * k) ||
            !in_periodic_box(J.P, x + 3 * k))
            return DEM_EINVAL;
    std::vector<Contact> c;
    dem_status r = read_contacts(s, slot, c);
    if (r != DEM_OK) return r;
    Job jd;
    r = read_job(s, slot, jd);
    if (r != DEM_OK) return r;
    Placed pl;
    place_job(J, x, v, w, pl);
    r = upload_job(s, slot, pl, jd.t, jd.steps_left);
    if (r != DEM_OK) return r;
    // keep the device time, step count and status
    r = upload(s, s->jobs_d[s->cur] + slot, &jd, sizeof(Job));
    if (r != DEM_OK) return r;
    HIPCHK(hipStreamSynchronize(s->stream));
    s->staging.clear();
    s->held.clear();
    return write_contacts(s, slot, c);
}

// New radii of a job's particles (pid order), keeping positions, velocities
// and contact history.  The grid stays: its cells must remain at least as
// wide as the largest contact distance, or, with the two-level search, as
// twice the radius cut (which this sets anew) and as the largest radius.  Masses and inertias follow the
// radii (they are computed from them in the kernels); the time step stays.
dem_status set_radii_impl(dem_pool* s, int slot, const float* radius) {
    HostJob& J = s->jobs[slot];
    const uint64_t n = J.n;
    double rmax = 0.0;
    for (uint64_t k = 0; k < n; ++k) {
        if (!(radius[k] > 0.0f) || !std::isfinite(radius[k])) return DEM_EINVAL;
        rmax = std::max(rmax, (double)radius[k]);
    }
    if (n == 0) return DEM_OK;
    // the cut the grid allows (the largest, so the fewest big particles):
    // pairs up to the cut within one cell, the largest radius within two
    double cmin = INFINITY;
    bool five = true;
    for (int a = 0; a < 3; ++a) {
        cmin = std::min(cmin, J.lay.cell[a]);
        if (((J.P.periodic >> a) & 1u) && J.lay.nc[a] < 5) five = false;
    }
    double used = std::min(rmax, 0.5 * cmin / 1.000001);
    if (!J.two_level || !five) used = rmax;
    if (used >= rmax) {
        if (!(2.0 * rmax * 1.000001 <= cmin)) return DEM_EINVAL;
        used = rmax;
    } else if (!(rmax * 1.000001 <= cmin)) {
        return DEM_EINVAL;
    }
    Job jd;
    dem_status r = read_job(s, slot, jd);
    if (r != DEM_OK) return r;
    double span = 0.0;
    for (int a = 0; a < 3; ++a) span = std::max(span, std::fabs(J.geo.lo[a]) + std::fabs(J.geo.hi[a]));
    set_cut(J.geo, used, rmax, span);
    jd.g.reach = J.geo.reach;
    jd.g.reach_big = J.geo.reach_big;
    jd.g.rcut = J.geo.rcut;
    jd.g.nbig = J.geo.nbig;
    // the radii travel through the sort's scratch keys (unused between steps)
    r = upload(s, s->keys_t, radius, n * sizeof(float));
    if (r == DEM_OK) r = upload(s, s->jobs_d[s->cur] + slot, &jd, sizeof(Job));
    if (r != DEM_OK) return r;
    const uint32_t p0 = J.tile0 * TILE;
    launch_set_radii(p0, (uint32_t)n, (const float*)s->keys_t, s->S[s->cur], s->srt[s->cur],
                     s->stream);
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(s->stream));
    s->staging.clear();
    s->held.clear();
    J.r.assign(radius, radius + n);
    return DEM_OK;
}

}  // namespace

// ======================================================================= ABI
extern "C" {

const char* dem_status_str(dem_status s) {
    switch (s) {
        case DEM_OK: return "ok";
        case DEM_EINVAL: return "invalid argument";
        case DEM_ENOMEM: return "out of memory";
        case DEM_ECAPACITY: return "contact capacity exceeded";
        case DEM_ENONFINITE: return "non-finite force or state";
        case DEM_EDEVICE: return "HIP runtime error";
        case DEM_EBUSY: return "pool full";
        case DEM_ESCRATCH: return "input too large for the static scratch";
    }
    return "unknown status";
}

uint64_t dem_footprint(const dem_params* P, uint64_t n) {
    if (!P) return 0;
    const uint64_t cells = std::max<uint64_t>(4 * n, 4096);
    const uint64_t np = std::max<uint64_t>(1, tiles_of(n)) * TILE;
    uint64_t slots = 8;
    if (P->max_contacts) slots = std::max<uint64_t>(1, (P->max_contacts + np - 1) / np);
    return pool_bytes(np / TILE, cells, 1, P->precision == DEM_PREC_FP64, slots, P->flags);
}

// ------------------------------------------------------- static scratch
// Device memory of the simulation dem_create_static makes: one array of
// DEM_STATIC_BYTES per device, reserved when the library's code object is
// loaded and held until the process ends.  In host code `scratch` only
// names the symbol; its device address on each device comes from
// hipGetSymbolAddress with that device current, and only that address is
// handed to kernels and copies (as the arena of the simulation).
static __device__ __align__(256) unsigned char scratch[DEM_STATIC_BYTES];

namespace {
constexpr int MAX_STATIC_DEVICES = 64;
std::mutex g_static_mu;
void* g_static_ptr[MAX_STATIC_DEVICES] = {};  // device address of scratch, per device
bool g_static_live[MAX_STATIC_DEVICES] = {};  // a simulation occupies that device's scratch

void release_static(int dev) {
    std::lock_guard<std::mutex> g(g_static_mu);
    g_static_live[dev] = false;
}
}  // namespace

dem_status dem_create(const dem_params* params, const dem_material* mats, uint32_t n_mats,
                      uint64_t n, const double* x, const double* v, const double* w,
                      const float* radius, const uint16_t* mat_id, void* device_arena,
                      uint64_t arena_bytes, void* stream, dem_sim** out) {
    if (!out) return DEM_EINVAL;
    *out = nullptr;
    dem_status r = validate(params, mats, n_mats);
    if (r != DEM_OK) return r;
    if (n >= (uint64_t)FACE) return DEM_EINVAL;
    if (n && (!x || !v || !w || !radius)) return DEM_EINVAL;
    // size the pool for exactly this job
    double rmax = 0.0;
    for (uint64_t i = 0; i < n; ++i)
        if (radius[i] > rmax) rmax = radius[i];
    if (n == 0 || !(rmax > 0.0) || !std::isfinite(rmax)) {
        double lmin = INFINITY;
        for (int a = 0; a < 3; ++a) lmin = std::min(lmin, params->hi[a] - params->lo[a]);
        rmax = lmin / 6.1;
    }
    Layout lay;
    double used = rmax;
    r = plan_job_grid(*params, rmax,
                      (n && half_search(params->flags)) ? radius_cut(*params, radius, n, rmax)
                                                        : rmax, n,
                      lay, used);
    if (r != DEM_OK) return r;
    const uint64_t np = std::max<uint64_t>(1, tiles_of(n)) * TILE;
    uint32_t slots = 8;
    if (params->max_contacts)
        slots = (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>((params->max_contacts + np - 1) / np, 1024));
    dem_pool* p = nullptr;
    if (device_arena && arena_bytes < dem_footprint(params, n)) return DEM_EINVAL;
    r = create_pool(n, (uint64_t)lay.nc[0] * lay.nc[1] * lay.nc[2], 1,
                    params->precision == DEM_PREC_FP64, slots, params->flags, device_arena,
                    arena_bytes, stream, &p);
    if (r != DEM_OK) return r;
    int slot = 0;
    Prepared pj;
    r = prepare_job(params, mats, n_mats, n, x, v, w, radius, mat_id, half_search(params->flags),
                    pj);
    if (r == DEM_OK) r = commit_job(p, pj, 0xFFFFFFFFu, &slot);
    if (r == DEM_OK) r = sync_impl(p);
    if (r != DEM_OK) {
        destroy_pool(p);
        return r == DEM_EBUSY ? DEM_EINVAL : r;
    }
    dem_sim* s = new (std::nothrow) dem_sim();
    if (!s) {
        destroy_pool(p);
        return DEM_ENOMEM;
    }
    s->pool = p;
    s->slot = slot;
    *out = s;
    return DEM_OK;
}

dem_status dem_create_static(const dem_params* params, const dem_material* mats,
                             uint32_t n_mats, uint64_t n, const double* x, const double* v,
                             const double* w, const float* radius, const uint16_t* mat_id,
                             void* stream, dem_sim** out) {
    if (!out || !params) return DEM_EINVAL;
    *out = nullptr;
    if (dem_footprint(params, n) > DEM_STATIC_BYTES) return DEM_ESCRATCH;
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_STATIC_DEVICES) return DEM_EDEVICE;
    void* base = nullptr;
    {
        std::lock_guard<std::mutex> g(g_static_mu);
        if (g_static_live[dev]) return DEM_EBUSY;
        if (!g_static_ptr[dev]) {
            void* p = nullptr;
            hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p) {
                (void)hipGetLastError();
                return DEM_EDEVICE;
            }
            g_static_ptr[dev] = p;
        }
        base = g_static_ptr[dev];
        g_static_live[dev] = true;  // held while this call builds the simulation
    }
    // the scratch keeps the previous simulation's contents: create_pool
    // clears every buffer that must start at zero, as it does for an arena
    dem_status r = dem_create(params, mats, n_mats, n, x, v, w, radius, mat_id, base,
                              DEM_STATIC_BYTES, stream, out);
    if (r != DEM_OK) {
        release_static(dev);
        return r;
    }
    (*out)->static_dev = dev;
    return DEM_OK;
}

dem_status dem_step(dem_sim* s, uint32_t nsteps) {
    if (!s) return DEM_EINVAL;
    return step_impl(s->pool, nsteps);
}

// A single simulation reports its job's non-finite failure as an error.
static dem_status sim_sync(dem_sim* s) {
    dem_status r = sync_impl(s->pool);
    if (r != DEM_OK) return r;
    Job jd;
    r = read_job(s->pool, s->slot, jd);
    if (r != DEM_OK) return r;
    return jd.status == JOB_FAILED ? DEM_ENONFINITE : DEM_OK;
}

dem_status dem_sync(dem_sim* s) {
    if (!s) return DEM_EINVAL;
    return sim_sync(s);
}

dem_status dem_get_state(dem_sim* s, double* x, double* v, double* w, double* F, double* T) {
    if (!s) return DEM_EINVAL;
    dem_status r = sim_sync(s);
    if (r != DEM_OK && r != DEM_ENONFINITE) return r;
    dem_status r2 = get_state_impl(s->pool, s->slot, x, v, w, F, T);
    return r2 != DEM_OK ? r2 : r;
}

dem_status dem_get_contacts(dem_sim* s, uint64_t cap, uint32_t* i, uint32_t* j, double* dt_xyz,
                            uint64_t* m) {
    if (!s || !m) return DEM_EINVAL;
    dem_status r = sim_sync(s);
    if (r != DEM_OK) return r;
    std::vector<Contact> c;
    r = read_contacts(s->pool, s->slot, c);
    if (r != DEM_OK) return r;
    *m = c.size();
    const uint64_t k = std::min<uint64_t>(cap, c.size());
    for (uint64_t q = 0; q < k; ++q) {
        if (i) i[q] = c[q].i;
        if (j) j[q] = c[q].j;
        if (dt_xyz)
            for (int a = 0; a < 3; ++a) dt_xyz[3 * q + a] = c[q].dt[a];
    }
    return DEM_OK;
}

dem_status dem_set_contacts(dem_sim* s, uint64_t m, const uint32_t* i, const uint32_t* j,
                            const double* dt_xyz) {
    if (!s) return DEM_EINVAL;
    if (m && (!i || !j || !dt_xyz)) return DEM_EINVAL;
    dem_status r = sim_sync(s);
    if (r != DEM_OK) return r;
    std::vector<Contact> c(m);
    for (uint64_t q = 0; q < m; ++q) {
        c[q].i = i[q];
        c[q].j = j[q];
        for (int a = 0; a < 3; ++a) c[q].dt[a] = dt_xyz[3 * q + a];
    }
    return write_contacts(s->pool, s->slot, c);
}

dem_status dem_set_state(dem_sim* s, const double* x, const double* v, const double* w) {
    if (!s || (s->pool->jobs[s->slot].n && (!x || !v || !w))) return DEM_EINVAL;
    dem_status r = sim_sync(s);
    if (r != DEM_OK) return r;
    return set_state_impl(s->pool, s->slot, x, v, w);
}

dem_status dem_set_radii(dem_sim* s, const float* radius) {
    if (!s || (s->pool->jobs[s->slot].n && !radius)) return DEM_EINVAL;
    dem_status r = sim_sync(s);
    if (r != DEM_OK) return r;
    return set_radii_impl(s->pool, s->slot, radius);
}

dem_status dem_get_info(dem_sim* s, dem_info* info) {
    if (!s || !info) return DEM_EINVAL;
    dem_pool* p = s->pool;
    dem_status r = sim_sync(s);
    if (r != DEM_OK && r != DEM_ENONFINITE) return r;
    Job jd;
    dem_status r2 = read_job(p, s->slot, jd);
    if (r2 != DEM_OK) return r2;
    const HostJob& J = p->jobs[s->slot];
    std::memset(info, 0, sizeof(*info));
    info->n = J.n;
    info->steps_done = jd.steps_done;
    info->dt = J.geo.dt;
    info->time = jd.t;
    info->capacity = (uint64_t)J.ntiles * TILE * p->slots;
    info->regrows = p->regrows;
    for (int a = 0; a < 3; ++a) info->cells[a] = (uint32_t)J.lay.nc[a];
    info->key_bits = (uint32_t)J.lay.key_bits;
    info->device_bytes = p->device_bytes;
    info->radius_cut = (double)J.geo.rcut;
    for (const float rr : J.r) info->big += rr > J.geo.rcut ? 1u : 0u;
    std::vector<TileStats> ts(J.ntiles);
    if (J.ntiles)
        HIPCHK(hipMemcpy(ts.data(), p->ts + J.tile0, J.ntiles * sizeof(TileStats), hipMemcpyDeviceToHost));
    for (const TileStats& q : ts) {
        info->sum_contacts += q.m;
        info->sum_matched += q.matched;
        info->sum_old += q.old;
    }
    if (J.n) {
        std::vector<uint2> rows(J.n);
        HIPCHK(hipMemcpy(rows.data(), p->rows[p->cur] + J.tile0 * TILE, J.n * sizeof(uint2),
                         hipMemcpyDeviceToHost));
        for (const uint2& q : rows) info->contacts += q.y;
    }
    return r;
}

void dem_destroy(dem_sim* s) {
    if (!s) return;
    destroy_pool(s->pool);
    if (s->static_dev >= 0) release_static(s->static_dev);
    delete s;
}

static dem_status profile_read_impl(dem_pool* s, double* ms, uint64_t* launches) {
    HIPCHK(hipStreamSynchronize(s->stream));
    for (int p = 0; p < DEM_NPHASE; ++p) {
        ms[p] = 0.0;
        launches[p] = 0;
    }
    for (size_t k = 0; k < s->prof_used; ++k) {
        for (int p = 0; p < DEM_NPHASE; ++p) {
            float t = 0.0f;
            if (hipEventElapsedTime(&t, s->prof_ev[k].e[p], s->prof_ev[k].e[p + 1]) == hipSuccess) {
                ms[p] += t;
                launches[p] += 1;
            }
        }
    }
    s->prof_used = 0;
    return DEM_OK;
}

dem_status dem_profile(dem_sim* s, int enable) {
    if (!s) return DEM_EINVAL;
    s->pool->prof = enable != 0;
    return DEM_OK;
}

dem_status dem_profile_read(dem_sim* s, double* ms, uint64_t* launches) {
    if (!s || !ms || !launches) return DEM_EINVAL;
    return profile_read_impl(s->pool, ms, launches);
}

// ------------------------------------------------------------------- pool
// The capacities a pool gets: as given, or, with max_particles = 0, the
// most particle positions whose footprint fits the budget (hbm_budget, else
// the arena's size) with 4 cells per position plus 4096 per job slot (the
// largest grid a job can take) and max_jobs slots (256 when 0).
static bool resolve_pool(const dem_pool_params* pp, uint64_t arena_bytes, uint64_t& P,
                         uint64_t& C, uint32_t& J, uint32_t& slots) {
    if (pp->precision != DEM_PREC_FP64 && pp->precision != DEM_PREC_MIXED) return false;
    if (pp->contact_slots > 1024) return false;
    slots = pp->contact_slots ? (uint32_t)pp->contact_slots : 8u;
    const bool fp64 = pp->precision == DEM_PREC_FP64;
    P = pp->max_particles;
    C = pp->max_cells;
    J = pp->max_jobs;
    if (P) return J >= 1 && C >= 1;
    const uint64_t B = pp->hbm_budget ? pp->hbm_budget : arena_bytes;
    if (!B) return false;
    if (!J) J = 256;
    auto cells = [&](uint64_t t) { return C ? C : 4 * t * TILE + 4096ull * J; };
    auto fits = [&](uint64_t t) { return pool_bytes(t, cells(t), J, fp64, slots, pp->flags) <= B; };
    if (!fits(1)) return false;
    uint64_t lo = 1, hi = 1;
    while (fits(hi) && hi * TILE * slots < MAX_ENTRIES) hi *= 2;
    while (hi - lo > 1) {
        const uint64_t mid = (lo + hi) / 2;
        if (fits(mid)) lo = mid;
        else hi = mid;
    }
    P = lo * TILE;
    C = cells(lo);
    return true;
}

uint64_t dem_pool_footprint(const dem_pool_params* pp) {
    if (!pp) return 0;
    uint64_t P, C;
    uint32_t J, slots;
    if (!resolve_pool(pp, 0, P, C, J, slots)) return 0;
    return pool_bytes(std::max<uint64_t>(1, tiles_of(P)), C, J, pp->precision == DEM_PREC_FP64,
                      slots, pp->flags);
}

dem_status dem_pool_create(const dem_pool_params* pp, void* device_arena, uint64_t arena_bytes,
                           void* stream, dem_pool** out) {
    if (!pp || !out) return DEM_EINVAL;
    *out = nullptr;
    uint64_t P, C;
    uint32_t J, slots;
    if (!resolve_pool(pp, device_arena ? arena_bytes : 0, P, C, J, slots)) return DEM_EINVAL;
    const uint64_t need = pool_bytes(std::max<uint64_t>(1, tiles_of(P)), C, J,
                                     pp->precision == DEM_PREC_FP64, slots, pp->flags);
    if (pp->hbm_budget && need > pp->hbm_budget) return DEM_EINVAL;
    if (device_arena && need > arena_bytes) return DEM_EINVAL;
    return create_pool(P, C, J, pp->precision == DEM_PREC_FP64, slots, pp->flags, device_arena,
                       arena_bytes, stream, out);
}

dem_status dem_pool_add(dem_pool* s, const dem_params* params, const dem_material* mats,
                        uint32_t n_mats, uint64_t n, const double* x, const double* v,
                        const double* w, const float* radius, const uint16_t* mat_id,
                        uint32_t steps, uint64_t* job) {
    if (!s || !job) return DEM_EINVAL;
    if (s->failed != DEM_OK) return s->failed;
    if (steps == 0 || steps == 0xFFFFFFFFu) return DEM_EINVAL;
    if (params && (params->precision == DEM_PREC_FP64) != s->fp64) return DEM_EINVAL;
    // host work first, while enqueued steps run; then the job is placed
    // between steps
    Prepared pj;
    dem_status r = prepare_job(params, mats, n_mats, n, x, v, w, radius, mat_id,
                               half_search(s->flags), pj);
    if (r != DEM_OK) return r;
    r = sync_impl(s);
    if (r != DEM_OK) return r;
    int slot = 0;
    r = commit_job(s, pj, steps, &slot);
    if (r != DEM_OK) return r;
    *job = s->jobs[slot].id;
    return DEM_OK;
}

struct dem_job_prep {
    Prepared pj;
    bool used = false;
};

dem_status dem_job_prepare(const dem_params* params, const dem_material* mats, uint32_t n_mats,
                           uint64_t n, const double* x, const double* v, const double* w,
                           const float* radius, const uint16_t* mat_id, dem_job_prep** out) {
    if (!out) return DEM_EINVAL;
    *out = nullptr;
    dem_job_prep* p = new (std::nothrow) dem_job_prep();
    if (!p) return DEM_ENOMEM;
    dem_status r = DEM_OK;
    try {
        r = prepare_job(params, mats, n_mats, n, x, v, w, radius, mat_id,
                        params && half_search(params->flags), p->pj);
    } catch (const std::bad_alloc&) {
        r = DEM_ENOMEM;
    }
    if (r != DEM_OK) {
        delete p;
        return r;
    }
    *out = p;
    return DEM_OK;
}

uint64_t dem_job_prep_cells(const dem_job_prep* p) { return p && !p->used ? p->pj.J.ncells : 0; }

dem_status dem_pool_add_prepared(dem_pool* s, dem_job_prep* p, uint32_t steps, uint64_t* job) {
    if (!s || !p || !job || p->used) return DEM_EINVAL;
    if (s->failed != DEM_OK) return s->failed;
    if (steps == 0 || steps == 0xFFFFFFFFu) return DEM_EINVAL;
    if ((p->pj.J.P.precision == DEM_PREC_FP64) != s->fp64) return DEM_EINVAL;
    // a job prepared for the two-level search needs the pool's half search
    if (p->pj.J.geo.nbig && !half_search(s->flags)) return DEM_EINVAL;
    dem_status r = sync_impl(s);
    if (r != DEM_OK) return r;
    int slot = 0;
    r = commit_job(s, p->pj, steps, &slot);
    if (r == DEM_EBUSY) return r;  // the prepared job stays usable
    p->used = true;
    if (r != DEM_OK) return r;
    *job = s->jobs[slot].id;
    return DEM_OK;
}

void dem_job_prep_free(dem_job_prep* p) { delete p; }

static int slot_of(dem_pool* s, uint64_t id) {
    for (uint32_t k = 0; k < s->max_jobs; ++k)
        if (s->jobs[k].used && s->jobs[k].id == id) return (int)k;
    return -1;
}

dem_status dem_pool_step(dem_pool* s, uint32_t nsteps) {
    if (!s) return DEM_EINVAL;
    return step_impl(s, nsteps);
}

dem_status dem_pool_sync(dem_pool* s) {
    if (!s) return DEM_EINVAL;
    return sync_impl(s);
}

dem_status dem_pool_poll(dem_pool* s, uint64_t* done, uint32_t cap, uint32_t* n_done) {
    if (!s || !n_done || (cap && !done)) return DEM_EINVAL;
    *n_done = 0;
    dem_status r = sync_impl(s);
    if (r != DEM_OK) return r;
    std::vector<Job> jd(s->max_jobs);
    HIPCHK(hipMemcpy(jd.data(), s->jobs_d[s->cur], s->max_jobs * sizeof(Job), hipMemcpyDeviceToHost));
    uint32_t k = 0;
    for (uint32_t q = 0; q < s->max_jobs && k < cap; ++q) {
        HostJob& J = s->jobs[q];
        if (!J.used || J.reported || jd[q].status == JOB_ACTIVE) continue;
        done[k++] = J.id;
        J.reported = true;
    }
    *n_done = k;
    return DEM_OK;
}

dem_status dem_pool_job_info(dem_pool* s, uint64_t job, dem_job_info* info) {
    if (!s || !info) return DEM_EINVAL;
    const int slot = slot_of(s, job);
    if (slot < 0) return DEM_EINVAL;
    dem_status r = sync_impl(s);
    if (r != DEM_OK) return r;
    Job jd;
    r = read_job(s, slot, jd);
    if (r != DEM_OK) return r;
    std::memset(info, 0, sizeof(*info));
    info->status = jd.status == JOB_ACTIVE ? DEM_JOB_RUNNING
                                           : (jd.status == JOB_DONE ? DEM_JOB_DONE : DEM_JOB_FAILED);
    info->n = s->jobs[slot].n;
    info->steps_done = jd.steps_done;
    info->steps_left = jd.steps_left;
    info->time = jd.t;
    info->dt = s->jobs[slot].geo.dt;
    return DEM_OK;
}

dem_status dem_pool_get_state(dem_pool* s, uint64_t job, double* x, double* v, double* w) {
    if (!s) return DEM_EINVAL;
    const int slot = slot_of(s, job);
    if (slot < 0) return DEM_EINVAL;
    dem_status r = sync_impl(s);
    if (r != DEM_OK) return r;
    return get_state_impl(s, slot, x, v, w, nullptr, nullptr);
}

dem_status dem_pool_set_radii(dem_pool* s, uint64_t job, const float* radius) {
    if (!s) return DEM_EINVAL;
    const int slot = slot_of(s, job);
    if (slot < 0 || (s->jobs[slot].n && !radius)) return DEM_EINVAL;
    dem_status r = sync_impl(s);
    if (r != DEM_OK) return r;
    return set_radii_impl(s, slot, radius);
}

dem_status dem_pool_remove(dem_pool* s, uint64_t job) {
    if (!s) return DEM_EINVAL;
    const int slot = slot_of(s, job);
    if (slot < 0) return DEM_EINVAL;
    dem_status r = sync_impl(s);
    if (r != DEM_OK) return r;
    return remove_job(s, slot);
}

uint64_t dem_job_cells(const dem_params* params, uint64_t n, double rmax) {
    if (!params || !(rmax > 0.0) || !std::isfinite(rmax)) return 0;
    Layout lay;
    double used = rmax;
    // the radius cut of the two-level search is at least rmax / 2: the grid
    // of that cut has the most cells a job can get
    if (plan_job_grid(*params, rmax, half_search(params->flags) ? 0.5 * rmax : rmax, n, lay,
                      used) != DEM_OK)
        return 0;
    return (uint64_t)lay.nc[0] * lay.nc[1] * lay.nc[2];
}

dem_status dem_pool_capacity(dem_pool* s, uint64_t* free_particles, uint64_t* free_cells,
                             uint32_t* free_jobs) {
    if (!s) return DEM_EINVAL;
    uint64_t best = 0, cells = 0;
    for (const Seg& g : s->segs)
        if (g.slot < 0) best = std::max<uint64_t>(best, (uint64_t)g.len * TILE);
    for (auto& f : s->free_cells) cells = std::max<uint64_t>(cells, f.second);
    uint32_t fj = 0;
    for (const HostJob& j : s->jobs) fj += j.used ? 0 : 1;
    if (free_particles) *free_particles = best;
    if (free_cells) *free_cells = cells;
    if (free_jobs) *free_jobs = fj;
    return DEM_OK;
}

dem_status dem_pool_profile(dem_pool* s, int enable) {
    if (!s) return DEM_EINVAL;
    s->prof = enable != 0;
    return DEM_OK;
}

dem_status dem_pool_profile_read(dem_pool* s, double* ms, uint64_t* launches) {
    if (!s || !ms || !launches) return DEM_EINVAL;
    return profile_read_impl(s, ms, launches);
}

void dem_pool_destroy(dem_pool* s) { destroy_pool(s); }

}  // extern "C"
