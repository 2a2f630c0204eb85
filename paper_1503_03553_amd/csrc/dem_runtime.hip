// Host runtime of libdem: validation, device memory, the step pipeline,
// capacity regrowth, state and contact-history transfer, and the C ABI
// declared in include/dem.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>
#include <vector>

#include "../../include/dem.h"
#include "dem_internal.h"

using namespace dem;

namespace {

constexpr double PI = 3.14159265358979323846;

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

struct Buf {
    void* p = nullptr;
    size_t bytes = 0;
};

struct ProfEv {
    hipEvent_t e[2 * DEM_NPHASE];
};

}  // namespace

struct dem_sim {
    dem_params P{};
    std::vector<dem_material> mats;
    uint64_t n = 0;
    hipStream_t stream = nullptr;
    int device = 0;
    bool fp64 = true;
    int kmax = 16;
    Geo geo{};
    double dt = 0.0;
    double time_done = 0.0;            // simulation time after the last confirmed step
    uint64_t steps_confirmed = 0;      // steps known to have completed
    uint64_t steps_enqueued = 0;
    std::vector<double> t_pending;     // start time of each enqueued, unconfirmed step
    uint32_t slots = 0;                // contact slots per particle of each tile's region
    uint64_t cap = 0;                  // ntiles * TILE * slots
    uint64_t regrows = 0;
    bool table_by_pid = true;          // old table indexed by pid (after create / set_contacts)
    dem_status failed = DEM_OK;
    std::vector<float> r;
    std::vector<uint16_t> mat;
    size_t ncells = 0;
    // device memory
    std::vector<Buf> bufs;
    State A{}, B{};
    uint2* cells = nullptr;
    uint2* rows[2] = {nullptr, nullptr};
    uint32_t* col_j = nullptr;
    uint32_t* tab_pid[2] = {nullptr, nullptr};
    double* tab_dt[2] = {nullptr, nullptr};
    uint32_t* prev = nullptr;
    uint32_t *keys = nullptr, *vals = nullptr, *keys_t = nullptr, *vals_t = nullptr;
    uint32_t* tile_hist = nullptr;
    uint32_t* digit_tot = nullptr;
    void* fo = nullptr;
    MatTable* mt = nullptr;
    Status* st = nullptr;
    TileStats* ts = nullptr;
    uint32_t ntiles = 0;
    size_t device_bytes = 0;
    // profiling
    bool prof = false;
    std::vector<ProfEv> prof_ev;
    size_t prof_used = 0;
};

namespace {

dem_status hip_status(hipError_t e) {
    if (e == hipSuccess) return DEM_OK;
    if (e == hipErrorOutOfMemory) return DEM_ENOMEM;
    return DEM_EDEVICE;
}

#define HIPCHK(x)                                   \
    do {                                            \
        hipError_t e_ = (x);                        \
        if (e_ != hipSuccess) return hip_status(e_); \
    } while (0)

dem_status dalloc(dem_sim* s, size_t bytes, void** out) {
    void* p = nullptr;
    if (bytes == 0) bytes = 256;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return DEM_ENOMEM;
    }
    s->bufs.push_back({p, bytes});
    s->device_bytes += bytes;
    *out = p;
    return DEM_OK;
}

void dfree(dem_sim* s, void* p) {
    if (!p) return;
    for (size_t k = 0; k < s->bufs.size(); ++k)
        if (s->bufs[k].p == p) {
            s->device_bytes -= s->bufs[k].bytes;
            s->bufs.erase(s->bufs.begin() + k);
            break;
        }
    (void)hipFree(p);
}

template <typename T>
dem_status dalloc_t(dem_sim* s, size_t count, T** out) {
    void* p;
    dem_status r = dalloc(s, count * sizeof(T), &p);
    if (r == DEM_OK) *out = (T*)p;
    return r;
}

double le_offset(const dem_sim* s, double t) {
    if (s->P.shear_rate == 0.0) return 0.0;
    const double Lx = s->P.hi[0] - s->P.lo[0], Ly = s->P.hi[1] - s->P.lo[1];
    const double u = s->P.shear_rate * Ly;
    return std::fmod(u * t, Lx);
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

struct Layout {
    int nc[3];
    double cell[3];
    int key_bits;
};

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
        int maxc = 1;
        for (int a = 0; a < 3; ++a) {
            const double L = P.hi[a] - P.lo[a];
            double c = std::floor(L / (want * 1.000001));
            if (c < 1) c = 1;
            if (c > 1024) c = 1024;
            out.nc[a] = (int)c;
            out.cell[a] = L / c;
            prod *= (uint64_t)c;
            maxc = std::max(maxc, (int)c);
        }
        if (prod > limit) {
            want *= 1.02;
            continue;
        }
        for (int a = 0; a < 3; ++a)
            if (((P.periodic >> a) & 1u) && out.nc[a] < 3) return DEM_EINVAL;
        int b = 0;
        while ((1 << b) < maxc) ++b;
        out.key_bits = 3 * b;
        return DEM_OK;
    }
    return DEM_EINVAL;
}

constexpr uint64_t MAX_ENTRIES = 0xFFFFFFF0ull;  // row starts are 32-bit

uint64_t tiles_of(uint64_t n) { return n ? (n + TILE - 1) / TILE : 1; }

dem_status alloc_contacts(dem_sim* s, uint32_t slots) {
    const uint64_t cap = tiles_of(s->n) * TILE * (uint64_t)slots;
    if (cap > MAX_ENTRIES) return DEM_ECAPACITY;
    dem_status r;
    if ((r = dalloc_t(s, cap, &s->col_j)) != DEM_OK) return r;
    for (int k = 0; k < 2; ++k) {
        if ((r = dalloc_t(s, cap, &s->tab_pid[k])) != DEM_OK) return r;
        if ((r = dalloc_t(s, 3 * (size_t)cap, &s->tab_dt[k])) != DEM_OK) return r;
    }
    s->cap = cap;
    s->slots = slots;
    return DEM_OK;
}

// Contact slots per particle: from max_contacts when given, else 8.
uint32_t initial_slots(const dem_params& P, uint64_t n) {
    if (P.max_contacts) {
        uint64_t sl = (P.max_contacts + tiles_of(n) * TILE - 1) / (tiles_of(n) * TILE);
        return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(sl, 1024));
    }
    return 8;
}

State state_view(void* xr, void* vw, void* mat) {
    State S;
    S.xr = (double4*)xr;
    S.vw = (double2*)vw;
    S.mat = (uint8_t*)mat;
    return S;
}

void set_step_geo(dem_sim* s, double t) {
    s->geo.le_shift = le_offset(s, t);
    s->geo.le_shift_next = le_offset(s, t + s->dt);
}

// Upload B (state in pid order), then hash, sort and reorder it into A.
dem_status upload_and_sort(dem_sim* s, const double* x, const double* v, const double* w) {
    const uint64_t n = s->n;
    if (n == 0) return DEM_OK;
    std::vector<double4> xr(n);
    std::vector<double2> vw(3 * n);
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t meta = pack_meta(s->r[i], (uint32_t)i);
        double mw;
        std::memcpy(&mw, &meta, 8);
        xr[i] = make_double4(x[3 * i], x[3 * i + 1], x[3 * i + 2], mw);
        vw[i] = make_double2(v[3 * i], v[3 * i + 1]);
        vw[n + i] = make_double2(v[3 * i + 2], w[3 * i]);
        vw[2 * n + i] = make_double2(w[3 * i + 1], w[3 * i + 2]);
    }
    HIPCHK(hipMemcpyAsync(s->B.xr, xr.data(), n * sizeof(double4), hipMemcpyHostToDevice, s->stream));
    HIPCHK(hipMemcpyAsync(s->B.vw, vw.data(), 3 * n * sizeof(double2), hipMemcpyHostToDevice, s->stream));
    if (s->B.mat) {
        std::vector<uint8_t> m8(n);
        for (uint64_t i = 0; i < n; ++i) m8[i] = (uint8_t)s->mat[i];
        HIPCHK(hipMemcpyAsync(s->B.mat, m8.data(), n, hipMemcpyHostToDevice, s->stream));
    }
    HIPCHK(hipMemsetAsync(s->cells, 0, s->ncells * sizeof(uint2), s->stream));
    launch_hash(s->B, (uint32_t)n, s->geo, s->keys, s->vals, s->stream);
    uint32_t *ko, *vo;
    launch_radix_sort(s->keys, s->vals, s->keys_t, s->vals_t, (uint32_t)n, s->geo.key_bits,
                      s->tile_hist, s->digit_tot, &ko, &vo, s->st, s->stream);
    launch_reorder(ko, vo, s->B, s->A, s->prev, s->cells, (uint32_t)n, s->geo, s->st, 0, s->stream);
    HIPCHK(hipGetLastError());
    // B now mirrors A's source order (pid order); keep F/T readable as zeros
    if (s->fo) HIPCHK(hipMemsetAsync(s->fo, 0, 6 * n * (s->fp64 ? 8 : 4), s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    return DEM_OK;
}

void prof_record(dem_sim* s, size_t step_slot, int ev) {
    if (!s->prof) return;
    (void)hipEventRecord(s->prof_ev[step_slot].e[ev], s->stream);
}

dem_status enqueue_step(dem_sim* s, uint64_t k, double t) {
    const uint32_t n = (uint32_t)s->n;
    set_step_geo(s, t);
    const int o = (int)(k & 1), w = 1 - o;
    size_t slot = 0;
    if (s->prof) {
        if (s->prof_used == s->prof_ev.size()) {
            ProfEv pe;
            for (int q = 0; q < 2 * DEM_NPHASE; ++q) HIPCHK(hipEventCreate(&pe.e[q]));
            s->prof_ev.push_back(pe);
        }
        slot = s->prof_used++;
    }
    prof_record(s, slot, 0);
    launch_detect(s->kmax, s->A, s->cells, n, s->geo, s->rows[w], s->col_j, s->slots, s->ts,
                  s->st, s->stream);
    prof_record(s, slot, 1);
    prof_record(s, slot, 2);
    launch_force(s->fp64, s->A, s->B, s->rows[w], s->col_j, s->rows[o], s->prev, s->tab_pid[o],
                 s->tab_dt[o], s->tab_pid[w], s->tab_dt[w], s->cap, s->cells, s->keys, s->vals,
                 (s->P.flags & DEM_FLAG_NO_FORCE_OUTPUT) ? nullptr : s->fo, s->mt, n, s->geo,
                 s->ts, s->st, s->stream);
    prof_record(s, slot, 3);
    prof_record(s, slot, 4);
    uint32_t *ko, *vo;
    launch_radix_sort(s->keys, s->vals, s->keys_t, s->vals_t, n, s->geo.key_bits, s->tile_hist,
                      s->digit_tot, &ko, &vo, s->st, s->stream);
    prof_record(s, slot, 5);
    prof_record(s, slot, 6);
    launch_reorder(ko, vo, s->B, s->A, s->prev, s->cells, n, s->geo, s->st, 1, s->stream);
    prof_record(s, slot, 7);
    HIPCHK(hipGetLastError());
    return DEM_OK;
}

dem_status read_status(dem_sim* s, Status& h) {
    HIPCHK(hipStreamSynchronize(s->stream));
    HIPCHK(hipMemcpy(&h, s->st, sizeof(Status), hipMemcpyDeviceToHost));
    return DEM_OK;
}

// Grow every tile's region of the contact table to hold `need` contacts per
// tile, keeping the old table of the step that is to be (re)run at the same
// positions (its rows hold absolute indices).
dem_status regrow(dem_sim* s, uint64_t need_per_tile, uint64_t step) {
    const uint64_t nt = tiles_of(s->n);
    uint64_t ns = std::max<uint64_t>((uint64_t)s->slots * 2, (need_per_tile + TILE - 1) / TILE + 2);
    if (nt * TILE * ns > MAX_ENTRIES) ns = MAX_ENTRIES / (nt * TILE);
    if (ns <= s->slots) return DEM_ECAPACITY;
    const uint64_t nc = nt * TILE * ns, oc = s->cap;
    uint32_t *col = nullptr, *pid[2] = {nullptr, nullptr};
    double* dt[2] = {nullptr, nullptr};
    bool ok = dalloc_t(s, nc, &col) == DEM_OK;
    for (int k = 0; k < 2 && ok; ++k)
        ok = dalloc_t(s, nc, &pid[k]) == DEM_OK && dalloc_t(s, 3 * nc, &dt[k]) == DEM_OK;
    if (!ok) {
        dfree(s, col);
        for (int k = 0; k < 2; ++k) {
            dfree(s, pid[k]);
            dfree(s, dt[k]);
        }
        return DEM_ECAPACITY;
    }
    const int o = (int)(step & 1);
    HIPCHK(hipMemcpyAsync(pid[o], s->tab_pid[o], oc * 4, hipMemcpyDeviceToDevice, s->stream));
    for (int c = 0; c < 3; ++c)
        HIPCHK(hipMemcpyAsync(dt[o] + (size_t)c * nc, s->tab_dt[o] + (size_t)c * oc, oc * 8,
                              hipMemcpyDeviceToDevice, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    dfree(s, s->col_j);
    for (int k = 0; k < 2; ++k) {
        dfree(s, s->tab_pid[k]);
        dfree(s, s->tab_dt[k]);
    }
    s->col_j = col;
    for (int k = 0; k < 2; ++k) {
        s->tab_pid[k] = pid[k];
        s->tab_dt[k] = dt[k];
    }
    s->cap = nc;
    s->slots = (uint32_t)ns;
    s->regrows++;
    return DEM_OK;
}

dem_status sync_impl(dem_sim* s) {
    if (s->failed != DEM_OK) return s->failed;
    for (;;) {
        Status h;
        dem_status r = read_status(s, h);
        if (r != DEM_OK) return r;
        const uint64_t done = h.steps_done;
        // confirm completed steps
        while (s->steps_confirmed < done) {
            s->time_done = s->t_pending.front() + s->dt;
            s->t_pending.erase(s->t_pending.begin());
            s->steps_confirmed++;
        }
        if (h.err == 0) return DEM_OK;
        if (h.err & ERR_NONFINITE) {
            s->failed = DEM_ENONFINITE;
            return DEM_ENONFINITE;
        }
        if (h.err & ERR_ROW) {
            if (s->kmax >= 64) {
                s->failed = DEM_ECAPACITY;
                return DEM_ECAPACITY;
            }
            s->kmax = 64;
        }
        if (h.err & ERR_CAPACITY) {
            r = regrow(s, h.need, done);
            if (r != DEM_OK) {
                s->failed = r;
                return r;
            }
        }
        // clear the error and the reservation counter, then redo the remaining steps
        Status z = h;
        z.err = 0;
        z.need = 0;
        HIPCHK(hipMemcpy(s->st, &z, sizeof(Status), hipMemcpyHostToDevice));
        s->prof_used = 0;
        std::vector<double> ts = s->t_pending;
        for (size_t q = 0; q < ts.size(); ++q) {
            r = enqueue_step(s, done + q, ts[q]);
            if (r != DEM_OK) return r;
        }
    }
}

void destroy_impl(dem_sim* s) {
    if (!s) return;
    (void)hipStreamSynchronize(s->stream);
    for (auto& b : s->bufs) (void)hipFree(b.p);
    s->bufs.clear();
    for (auto& pe : s->prof_ev)
        for (int q = 0; q < 2 * DEM_NPHASE; ++q) (void)hipEventDestroy(pe.e[q]);
    delete s;
}

bool finite3(const double* p) { return std::isfinite(p[0]) && std::isfinite(p[1]) && std::isfinite(p[2]); }

// pid of the particle at each position of B (the order of the last step's rows)
dem_status pids_of_B(dem_sim* s, std::vector<uint32_t>& pid) {
    const uint64_t n = s->n;
    std::vector<double4> xr(n);
    pid.resize(n);
    if (n) HIPCHK(hipMemcpy(xr.data(), s->B.xr, n * sizeof(double4), hipMemcpyDeviceToHost));
    for (uint64_t i = 0; i < n; ++i) {
        uint64_t m;
        std::memcpy(&m, &xr[i].w, 8);
        pid[i] = (uint32_t)(m >> 32);
    }
    return DEM_OK;
}

struct Contact {
    uint32_t i, j;
    double dt[3];
};

dem_status read_contacts(dem_sim* s, std::vector<Contact>& out) {
    out.clear();
    const uint64_t n = s->n;
    if (n == 0) return DEM_OK;
    const int o = (int)(s->steps_confirmed & 1);
    std::vector<uint2> rows(n);
    HIPCHK(hipMemcpy(rows.data(), s->rows[o], n * sizeof(uint2), hipMemcpyDeviceToHost));
    uint64_t m = 0;
    for (auto& r : rows) m = std::max<uint64_t>(m, (uint64_t)r.x + r.y);
    std::vector<uint32_t> tp(m);
    std::vector<double> td(3 * m);
    if (m) {
        HIPCHK(hipMemcpy(tp.data(), s->tab_pid[o], m * 4, hipMemcpyDeviceToHost));
        for (int c = 0; c < 3; ++c)
            HIPCHK(hipMemcpy(td.data() + c * m, s->tab_dt[o] + (size_t)c * s->cap, m * 8,
                             hipMemcpyDeviceToHost));
    }
    std::vector<uint32_t> pid;
    if (s->table_by_pid) {
        pid.resize(n);
        std::iota(pid.begin(), pid.end(), 0u);
    } else {
        dem_status r = pids_of_B(s, pid);
        if (r != DEM_OK) return r;
    }
    for (uint64_t p = 0; p < n; ++p)
        for (uint32_t k = rows[p].x; k < rows[p].x + rows[p].y; ++k)
            out.push_back({pid[p], tp[k], {td[k], td[m + k], td[2 * m + k]}});
    std::sort(out.begin(), out.end(), [](const Contact& a, const Contact& b) {
        return a.i < b.i || (a.i == b.i && a.j < b.j);
    });
    return DEM_OK;
}

// Install a history indexed by pid as the old table of the next step.
dem_status write_contacts(dem_sim* s, std::vector<Contact>& c) {
    const uint64_t n = s->n;
    std::sort(c.begin(), c.end(), [](const Contact& a, const Contact& b) {
        return a.i < b.i || (a.i == b.i && a.j < b.j);
    });
    for (size_t k = 0; k < c.size(); ++k) {
        if (c[k].i >= n) return DEM_EINVAL;
        if (c[k].j >= n && c[k].j < FACE) return DEM_EINVAL;
        if (c[k].j >= FACE + 6) return DEM_EINVAL;
        if (c[k].j == c[k].i) return DEM_EINVAL;
        if (k && c[k].i == c[k - 1].i && c[k].j == c[k - 1].j) return DEM_EINVAL;
        if (!finite3(c[k].dt)) return DEM_EINVAL;
    }
    while (c.size() > s->cap) {
        dem_status r = regrow(s, (c.size() + tiles_of(n) - 1) / tiles_of(n), s->steps_confirmed);
        if (r != DEM_OK) return r;
    }
    const int o = (int)(s->steps_confirmed & 1);
    const size_t m = c.size();
    std::vector<uint2> rows(n, make_uint2(0, 0));
    std::vector<uint32_t> tp(m);
    std::vector<double> td(3 * std::max<size_t>(m, 1));
    for (size_t k = 0; k < m; ++k) {
        if (rows[c[k].i].y == 0) rows[c[k].i].x = (uint32_t)k;
        rows[c[k].i].y++;
        tp[k] = c[k].j;
        for (int a = 0; a < 3; ++a) td[a * m + k] = c[k].dt[a];
    }
    if (n) HIPCHK(hipMemcpy(s->rows[o], rows.data(), n * sizeof(uint2), hipMemcpyHostToDevice));
    if (m) {
        HIPCHK(hipMemcpy(s->tab_pid[o], tp.data(), m * 4, hipMemcpyHostToDevice));
        for (int a = 0; a < 3; ++a)
            HIPCHK(hipMemcpy(s->tab_dt[o] + (size_t)a * s->cap, td.data() + a * m, m * 8,
                             hipMemcpyHostToDevice));
    }
    // prev[i] = pid of the particle now at sorted position i
    if (n) {
        std::vector<double4> xr(n);
        HIPCHK(hipMemcpy(xr.data(), s->A.xr, n * sizeof(double4), hipMemcpyDeviceToHost));
        std::vector<uint32_t> pv(n);
        for (uint64_t i = 0; i < n; ++i) {
            uint64_t mm;
            std::memcpy(&mm, &xr[i].w, 8);
            pv[i] = (uint32_t)(mm >> 32);
        }
        HIPCHK(hipMemcpy(s->prev, pv.data(), n * 4, hipMemcpyHostToDevice));
    }
    s->table_by_pid = true;
    return DEM_OK;
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
        case DEM_EBUSY: return "busy";
    }
    return "unknown status";
}

uint64_t dem_footprint(const dem_params* P, uint64_t n) {
    if (!P) return 0;
    const uint64_t cells = std::max<uint64_t>(4 * n, 4096);  // the grid's upper bound
    const uint64_t cap = tiles_of(n) * TILE * (uint64_t)initial_slots(*P, n);
    const bool f64 = P->precision == DEM_PREC_FP64;
    const uint64_t nn = n ? n : 1;
    uint64_t b = 0;
    b += 2 * nn * (32 + 48 + 1);        // sorted state and integrated state
    b += 2 * nn * 8;                    // contact rows, two steps
    b += 5 * nn * 4;                    // prev, keys and values (two buffers)
    b += 6 * nn * (f64 ? 8 : 4);        // per-particle F, T
    b += cells * 8;                     // cell bounds
    b += cap * (4 + 2 * 28);            // partner list and two history tables
    b += sort_hist_words((uint32_t)nn) * 4 + 256 * 4 + sizeof(MatTable) + sizeof(Status);
    b += tiles_of(n) * sizeof(TileStats);
    return b;
}

dem_status dem_create(const dem_params* params, const dem_material* mats, uint32_t n_mats,
                      uint64_t n, const double* x, const double* v, const double* w,
                      const float* radius, const uint16_t* mat_id, void* stream, dem_sim** out) {
    if (!out) return DEM_EINVAL;
    *out = nullptr;
    dem_status r = validate(params, mats, n_mats);
    if (r != DEM_OK) return r;
    if (n >= (uint64_t)FACE) return DEM_EINVAL;
    if (n && (!x || !v || !w || !radius)) return DEM_EINVAL;
    double rmax = 0.0;
    for (uint64_t i = 0; i < n; ++i) {
        if (!(radius[i] > 0.0f) || !std::isfinite(radius[i])) return DEM_EINVAL;
        if (!finite3(x + 3 * i) || !finite3(v + 3 * i) || !finite3(w + 3 * i)) return DEM_EINVAL;
        if (mat_id && mat_id[i] >= n_mats) return DEM_EINVAL;
        rmax = std::max(rmax, (double)radius[i]);
    }
    dem_sim* s = new (std::nothrow) dem_sim();
    if (!s) return DEM_ENOMEM;
    s->P = *params;
    s->mats.assign(mats, mats + n_mats);
    s->n = n;
    s->stream = (hipStream_t)stream;
    (void)hipGetDevice(&s->device);
    s->fp64 = params->precision == DEM_PREC_FP64;
    s->r.assign(radius, radius + n);
    s->mat.assign(n, 0);
    if (mat_id) s->mat.assign(mat_id, mat_id + n);
    const bool multi = n_mats > 1;

    Layout lay;
    if (n == 0) {
        // no particles: any grid with 3 cells per axis will do
        double lmin = INFINITY;
        for (int a = 0; a < 3; ++a) lmin = std::min(lmin, params->hi[a] - params->lo[a]);
        rmax = lmin / 6.1;
    }
    r = plan_grid(*params, rmax, n, lay);
    if (r != DEM_OK) {
        delete s;
        return r;
    }
    Geo& G = s->geo;
    for (int a = 0; a < 3; ++a) {
        G.lo[a] = params->lo[a];
        G.hi[a] = params->hi[a];
        G.L[a] = params->hi[a] - params->lo[a];
        G.inv_cell[a] = 1.0 / lay.cell[a];
        G.nc[a] = lay.nc[a];
        G.g[a] = params->gravity[a];
    }
    G.walls = params->walls;
    G.periodic = params->periodic;
    G.le = params->shear_rate != 0.0;
    G.key_bits = lay.key_bits;
    G.le_dv = params->shear_rate * G.L[1];
    s->ncells = (size_t)lay.nc[0] * lay.nc[1] * lay.nc[2];

    MatTable mt;
    fill_mat_table(*params, s->mats, mt);
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
            const double rk = (double)radius[k];
            const double mk = mt.mass_pref[m] * rk * rk * rk;
            const double kn = mt.kn_pref[m * MAXMAT + m] * std::sqrt(rk * rk / (rk + rk));
            dt = hertz_contact_time(0.5 * mk, kn, 0.1) / 50.0;
        }
    }
    s->dt = dt;
    G.dt = dt;
    s->time_done = params->time;

    const size_t nn = n ? n : 1;
    void *xa, *va, *xb, *vb, *ma = nullptr, *mb = nullptr;
#define ALLOC_OR_FAIL(call)      \
    do {                         \
        r = (call);              \
        if (r != DEM_OK) {       \
            destroy_impl(s);     \
            return r;            \
        }                        \
    } while (0)
    ALLOC_OR_FAIL(dalloc(s, nn * sizeof(double4), &xa));
    ALLOC_OR_FAIL(dalloc(s, 3 * nn * sizeof(double2), &va));
    ALLOC_OR_FAIL(dalloc(s, nn * sizeof(double4), &xb));
    ALLOC_OR_FAIL(dalloc(s, 3 * nn * sizeof(double2), &vb));
    if (multi) {
        ALLOC_OR_FAIL(dalloc(s, nn, &ma));
        ALLOC_OR_FAIL(dalloc(s, nn, &mb));
    }
    s->A = state_view(xa, va, ma);
    s->B = state_view(xb, vb, mb);
    ALLOC_OR_FAIL(dalloc_t(s, s->ncells, &s->cells));
    ALLOC_OR_FAIL(dalloc_t(s, nn, &s->rows[0]));
    ALLOC_OR_FAIL(dalloc_t(s, nn, &s->rows[1]));
    ALLOC_OR_FAIL(dalloc_t(s, nn, &s->prev));
    ALLOC_OR_FAIL(dalloc_t(s, nn, &s->keys));
    ALLOC_OR_FAIL(dalloc_t(s, nn, &s->vals));
    ALLOC_OR_FAIL(dalloc_t(s, nn, &s->keys_t));
    ALLOC_OR_FAIL(dalloc_t(s, nn, &s->vals_t));
    ALLOC_OR_FAIL(dalloc_t(s, sort_hist_words((uint32_t)nn), &s->tile_hist));
    ALLOC_OR_FAIL(dalloc_t(s, 256, &s->digit_tot));
    ALLOC_OR_FAIL(dalloc(s, 6 * nn * (s->fp64 ? 8 : 4), &s->fo));
    ALLOC_OR_FAIL(dalloc_t(s, 1, &s->mt));
    ALLOC_OR_FAIL(dalloc_t(s, 1, &s->st));
    s->ntiles = (uint32_t)tiles_of(n);
    ALLOC_OR_FAIL(dalloc_t(s, s->ntiles, &s->ts));
    ALLOC_OR_FAIL(alloc_contacts(s, initial_slots(*params, n)));
#undef ALLOC_OR_FAIL
    hipError_t e = hipMemcpy(s->mt, &mt, sizeof(MatTable), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(s->st, 0, sizeof(Status));
    if (e == hipSuccess) e = hipMemset(s->ts, 0, s->ntiles * sizeof(TileStats));
    if (e == hipSuccess) e = hipMemset(s->rows[0], 0, nn * sizeof(uint2));
    if (e == hipSuccess) e = hipMemset(s->rows[1], 0, nn * sizeof(uint2));
    if (e != hipSuccess) {
        destroy_impl(s);
        return hip_status(e);
    }
    r = upload_and_sort(s, x, v, w);
    if (r != DEM_OK) {
        destroy_impl(s);
        return r;
    }
    *out = s;
    return DEM_OK;
}

dem_status dem_step(dem_sim* s, uint32_t nsteps) {
    if (!s) return DEM_EINVAL;
    if (s->failed != DEM_OK) return s->failed;
    double t = s->t_pending.empty() ? s->time_done : s->t_pending.back() + s->dt;
    for (uint32_t q = 0; q < nsteps; ++q) {
        s->t_pending.push_back(t);
        dem_status r = enqueue_step(s, s->steps_enqueued, t);
        if (r != DEM_OK) return r;
        s->steps_enqueued++;
        t = t + s->dt;
    }
    if (nsteps) s->table_by_pid = false;
    return DEM_OK;
}

dem_status dem_sync(dem_sim* s) {
    if (!s) return DEM_EINVAL;
    return sync_impl(s);
}

dem_status dem_get_state(dem_sim* s, double* x, double* v, double* w, double* F, double* T) {
    if (!s) return DEM_EINVAL;
    dem_status r = sync_impl(s);
    if (r != DEM_OK && r != DEM_ENONFINITE) return r;
    const uint64_t n = s->n;
    if (n == 0) return r;
    std::vector<double4> xr(n);
    std::vector<double2> vw(3 * n);
    HIPCHK(hipMemcpy(xr.data(), s->A.xr, n * sizeof(double4), hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(vw.data(), s->A.vw, 3 * n * sizeof(double2), hipMemcpyDeviceToHost));
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
            v[3 * p] = vw[i].x;
            v[3 * p + 1] = vw[i].y;
            v[3 * p + 2] = vw[n + i].x;
        }
        if (w) {
            w[3 * p] = vw[n + i].y;
            w[3 * p + 1] = vw[2 * n + i].x;
            w[3 * p + 2] = vw[2 * n + i].y;
        }
    }
    if (F || T) {
        std::vector<uint32_t> pid;
        dem_status r2 = pids_of_B(s, pid);
        if (r2 != DEM_OK) return r2;
        std::vector<double> f(6 * n);
        if (s->fp64) {
            HIPCHK(hipMemcpy(f.data(), s->fo, 6 * n * 8, hipMemcpyDeviceToHost));
        } else {
            std::vector<float> ff(6 * n);
            HIPCHK(hipMemcpy(ff.data(), s->fo, 6 * n * 4, hipMemcpyDeviceToHost));
            for (size_t k = 0; k < 6 * n; ++k) f[k] = ff[k];
        }
        for (uint64_t i = 0; i < n; ++i) {
            const uint32_t p = pid[i];
            for (int a = 0; a < 3; ++a) {
                if (F) F[3 * p + a] = f[a * n + i];
                if (T) T[3 * p + a] = f[(3 + a) * n + i];
            }
        }
    }
    return r;
}

dem_status dem_get_contacts(dem_sim* s, uint64_t cap, uint32_t* i, uint32_t* j, double* dt_xyz,
                            uint64_t* m) {
    if (!s || !m) return DEM_EINVAL;
    dem_status r = sync_impl(s);
    if (r != DEM_OK) return r;
    std::vector<Contact> c;
    r = read_contacts(s, c);
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
    dem_status r = sync_impl(s);
    if (r != DEM_OK) return r;
    std::vector<Contact> c(m);
    for (uint64_t q = 0; q < m; ++q) {
        c[q].i = i[q];
        c[q].j = j[q];
        for (int a = 0; a < 3; ++a) c[q].dt[a] = dt_xyz[3 * q + a];
    }
    return write_contacts(s, c);
}

dem_status dem_set_state(dem_sim* s, const double* x, const double* v, const double* w) {
    if (!s || (s->n && (!x || !v || !w))) return DEM_EINVAL;
    dem_status r = sync_impl(s);
    if (r != DEM_OK) return r;
    for (uint64_t k = 0; k < s->n; ++k)
        if (!finite3(x + 3 * k) || !finite3(v + 3 * k) || !finite3(w + 3 * k)) return DEM_EINVAL;
    std::vector<Contact> c;
    r = read_contacts(s, c);
    if (r != DEM_OK) return r;
    r = upload_and_sort(s, x, v, w);
    if (r != DEM_OK) return r;
    return write_contacts(s, c);
}

dem_status dem_get_info(dem_sim* s, dem_info* info) {
    if (!s || !info) return DEM_EINVAL;
    dem_status r = sync_impl(s);
    Status h;
    dem_status r2 = read_status(s, h);
    if (r2 != DEM_OK) return r2;
    std::memset(info, 0, sizeof(*info));
    info->n = s->n;
    info->steps_done = h.steps_done;
    info->dt = s->dt;
    info->time = s->time_done;
    std::vector<TileStats> ts(s->ntiles);
    HIPCHK(hipMemcpy(ts.data(), s->ts, s->ntiles * sizeof(TileStats), hipMemcpyDeviceToHost));
    for (const TileStats& q : ts) {
        info->sum_contacts += q.m;
        info->sum_matched += q.matched;
        info->sum_old += q.old;
    }
    if (s->n) {
        std::vector<uint2> rows(s->n);
        HIPCHK(hipMemcpy(rows.data(), s->rows[s->steps_confirmed & 1], s->n * sizeof(uint2),
                         hipMemcpyDeviceToHost));
        for (const uint2& q : rows) info->contacts += q.y;
    }
    info->capacity = s->cap;
    info->regrows = s->regrows;
    for (int a = 0; a < 3; ++a) info->cells[a] = (uint32_t)s->geo.nc[a];
    info->key_bits = (uint32_t)s->geo.key_bits;
    info->device_bytes = s->device_bytes;
    return r;
}

void dem_destroy(dem_sim* s) { destroy_impl(s); }

dem_status dem_profile(dem_sim* s, int enable) {
    if (!s) return DEM_EINVAL;
    s->prof = enable != 0;
    return DEM_OK;
}

dem_status dem_profile_read(dem_sim* s, double* ms, uint64_t* launches) {
    if (!s || !ms || !launches) return DEM_EINVAL;
    HIPCHK(hipStreamSynchronize(s->stream));
    for (int p = 0; p < DEM_NPHASE; ++p) {
        ms[p] = 0.0;
        launches[p] = 0;
    }
    for (size_t k = 0; k < s->prof_used; ++k) {
        for (int p = 0; p < DEM_NPHASE; ++p) {
            float t = 0.0f;
            if (hipEventElapsedTime(&t, s->prof_ev[k].e[2 * p], s->prof_ev[k].e[2 * p + 1]) == hipSuccess) {
                ms[p] += t;
                launches[p] += 1;
            }
        }
    }
    s->prof_used = 0;
    return DEM_OK;
}

}  // extern "C"
