// HIP kernels of one DEM step for CDNA4 (gfx950, wave64).
//
// Step = detect -> force -> radix sort -> reorder, all on one stream:
//
//  detect   one lane per particle scans the 27 cells around it (section 3.3,
//           "cell-based method"), keeps the partners it touches in an LDS row
//           ordered by partner id, and the workgroup reserves one contiguous
//           range of the contact list for its 128 particles.  This is the
//           paper's first loop (section 3.4: collect the ids of touching
//           partners first); the reservation compacts the rows device-wide,
//           so the next kernel sees only real contacts.
//  force    one lane per compacted contact: history match against the
//           previous step's table, the contact law (Eq. 1-4, torque), then a
//           per-particle sum in ascending partner id through LDS, gravity
//           ("ForceGravity"), semi-implicit Euler ("Integrate"), and the new
//           cell key ("CalcHash").  This is the paper's second loop, with
//           every lane of a wavefront busy on a real contact.
//  sort     LSD radix sort of the cell keys ("BitonicSort" in the paper),
//           8-bit digits, reduce-then-scan, wave64 ballot ranking.
//  reorder  gathers the state into the new cell order and writes the cell
//           bounds ("FindCellBoundsAndReorder").
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "dem_internal.h"

namespace dem {

// ------------------------------------------------------------------ helpers
__device__ inline uint32_t xcd_tile(uint32_t b, uint32_t nb) {
    // Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
    // contiguous run of tiles so that neighbouring tiles share its L2.
    uint32_t q = nb >> 3, rem = nb & 7u, x = b & 7u, k = b >> 3;
    uint32_t start = x < rem ? x * (q + 1) : rem * (q + 1) + (x - rem) * q;
    return start + k;
}

__device__ inline float meta_r(double w) {
    return __uint_as_float((uint32_t)__double_as_longlong(w));
}
__device__ inline uint32_t meta_pid(double w) {
    return (uint32_t)((unsigned long long)__double_as_longlong(w) >> 32);
}

__device__ inline int cell_coord(const Geo& G, double x, int a) {
    double f = floor((x - G.lo[a]) * G.inv_cell[a]);
    if (!(f >= 0.0)) return 0;  // also NaN
    if (f >= (double)G.nc[a]) return G.nc[a] - 1;
    return (int)f;
}

__device__ inline uint32_t spread3(uint32_t v) {
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}
__device__ inline uint32_t compact3(uint32_t v) {
    v &= 0x09249249u;
    v = (v ^ (v >> 2)) & 0x030C30C3u;
    v = (v ^ (v >> 4)) & 0x0300F00Fu;
    v = (v ^ (v >> 8)) & 0xFF0000FFu;
    v = (v ^ (v >> 16)) & 0x000003FFu;
    return v;
}
__device__ inline uint32_t morton(int cx, int cy, int cz) {
    return spread3((uint32_t)cx) | (spread3((uint32_t)cy) << 1) | (spread3((uint32_t)cz) << 2);
}
__device__ inline uint32_t cell_key(const Geo& G, double x, double y, double z) {
    return morton(cell_coord(G, x, 0), cell_coord(G, y, 1), cell_coord(G, z, 2));
}
__device__ inline uint32_t key_lin(const Geo& G, uint32_t key) {
    uint32_t cx = compact3(key), cy = compact3(key >> 1), cz = compact3(key >> 2);
    return (cz * (uint32_t)G.nc[1] + cy) * (uint32_t)G.nc[0] + cx;
}

// Image of partner j that can touch i: periodic copies by minimum image, the
// Lees-Edwards copy across y carrying the shear offset along x.  Returns the
// shift S added to the raw difference x_j - x_i and the y-image index.
__device__ inline void image_shift(const Geo& G, double dx, double dy, double dz, double& Sx,
                                   double& Sy, double& Sz, int& ky) {
    ky = 0;
    Sx = Sy = Sz = 0.0;
    if (G.periodic & 2u) {
        ky = -(int)rint(dy / G.L[1]);
        Sy = (double)ky * G.L[1];
    }
    if (G.periodic & 1u) {
        double dxp = dx + (double)ky * G.le_shift;
        int kx = -(int)rint(dxp / G.L[0]);
        Sx = (double)kx * G.L[0] + (double)ky * G.le_shift;
    }
    if (G.periodic & 4u) {
        int kz = -(int)rint(dz / G.L[2]);
        Sz = (double)kz * G.L[2];
    }
}

// The contact predicate on FP64 positions, written out with no fused
// multiply-add so that the contact set is bit-exact: ((dx^2+dy^2)+dz^2) < s^2.
__device__ inline bool touching(double dx, double dy, double dz, double s) {
#pragma clang fp contract(off)
    double d2 = dx * dx + dy * dy;
    d2 = d2 + dz * dz;
    return d2 < s * s;
}

__device__ inline uint32_t skip_if_error(const Status* st, uint32_t* s_flag) {
    if (threadIdx.x == 0) *s_flag = __atomic_load_n(&st->err, __ATOMIC_RELAXED);
    __syncthreads();
    return *s_flag;
}

// Exclusive scan of v over the workgroup (blockDim = TILE = 2 waves).
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* s_w, uint32_t& total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t u = __shfl_up(x, o, 64);
        if (lane >= o) x += u;
    }
    if (lane == 63) s_w[w] = x;
    __syncthreads();
    uint32_t off = (w == 1) ? s_w[0] : 0u;
    total = s_w[0] + s_w[1];
    return x - v + off;
}

// Largest o in [0, TILE) with e[o] <= q, for e non-decreasing with e[0] = 0.
__device__ inline int owner_of(const uint32_t* e, uint32_t q) {
    int lo = 0, hi = TILE;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (e[mid] <= q) lo = mid;
        else hi = mid;
    }
    return lo;
}

// ------------------------------------------------------------------ detect
template <int KMAX>
__global__ __launch_bounds__(TILE) void k_detect(const double4* __restrict__ xr,
                                                 const uint2* __restrict__ cells, uint32_t n,
                                                 Geo G, uint2* __restrict__ rows,
                                                 uint32_t* __restrict__ col_j, uint32_t slots,
                                                 TileStats* __restrict__ ts, Status* st) {
    __shared__ uint32_t s_pid[KMAX * TILE];
    __shared__ uint32_t s_j[KMAX * TILE];
    __shared__ uint32_t s_excl[TILE + 1];
    __shared__ uint32_t s_w[2];
    __shared__ uint32_t s_base, s_flag;
    if (skip_if_error(st, &s_flag)) return;

    const int t = threadIdx.x;
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t i = tile * TILE + t;
    uint32_t cnt = 0;
    if (i < n) {
        const double4 a = xr[i];
        const double ri = (double)meta_r(a.w);
        const int cx = cell_coord(G, a.x, 0), cy = cell_coord(G, a.y, 1), cz = cell_coord(G, a.z, 2);
        for (int oz = -1; oz <= 1; ++oz) {
            int qz = cz + oz;
            if (qz < 0 || qz >= G.nc[2]) {
                if (!(G.periodic & 4u)) continue;
                qz = qz < 0 ? qz + G.nc[2] : qz - G.nc[2];
            }
            for (int oy = -1; oy <= 1; ++oy) {
                int qy = cy + oy, kyc = 0;
                if (qy < 0 || qy >= G.nc[1]) {
                    if (!(G.periodic & 2u)) continue;
                    kyc = qy < 0 ? -1 : 1;
                    qy -= kyc * G.nc[1];
                }
                // across a sheared y boundary the partner row is offset along x
                int cxq = cx;
                if (G.le && kyc != 0) {
                    double fx = floor((a.x - (double)kyc * G.le_shift - G.lo[0]) * G.inv_cell[0]);
                    const double lim = 2.0 * (double)G.nc[0];
                    if (!(fx >= -lim)) fx = -lim;  // also NaN
                    if (fx > lim) fx = lim;
                    cxq = (int)fx;
                }
                for (int ox = -1; ox <= 1; ++ox) {
                    int qx = cxq + ox;
                    if (qx < 0 || qx >= G.nc[0]) {
                        if (!(G.periodic & 1u)) continue;
                        qx %= G.nc[0];
                        if (qx < 0) qx += G.nc[0];
                    }
                    const uint2 rg = cells[(qz * G.nc[1] + qy) * G.nc[0] + qx];
                    for (uint32_t j = rg.x; j < rg.y; ++j) {
                        if (j == i) continue;
                        const double4 b = xr[j];
                        double dx = b.x - a.x, dy = b.y - a.y, dz = b.z - a.z;
                        if (G.periodic) {
                            double Sx, Sy, Sz;
                            int ky;
                            image_shift(G, dx, dy, dz, Sx, Sy, Sz, ky);
                            dx = dx + Sx;
                            dy = dy + Sy;
                            dz = dz + Sz;
                        }
                        const double s = ri + (double)meta_r(b.w);
                        if (touching(dx, dy, dz, s)) {
                            if (cnt < KMAX) {
                                const uint32_t pj = meta_pid(b.w);
                                int k = (int)cnt;
                                while (k > 0 && s_pid[(k - 1) * TILE + t] > pj) {
                                    s_pid[k * TILE + t] = s_pid[(k - 1) * TILE + t];
                                    s_j[k * TILE + t] = s_j[(k - 1) * TILE + t];
                                    --k;
                                }
                                s_pid[k * TILE + t] = pj;
                                s_j[k * TILE + t] = j;
                            }
                            ++cnt;
                        }
                    }
                }
            }
        }
        // box faces last, in face order (their ids sort after every particle)
        if (G.walls) {
            const double p[3] = {a.x, a.y, a.z};
            for (int f = 0; f < 6; ++f) {
                if (!(G.walls & (1u << f))) continue;
                const int ax = f >> 1;
                const double dist = (f & 1) ? G.hi[ax] - p[ax] : p[ax] - G.lo[ax];
                if (dist < ri) {
                    if (cnt < KMAX) {
                        s_pid[cnt * TILE + t] = FACE + (uint32_t)f;
                        s_j[cnt * TILE + t] = FACE + (uint32_t)f;
                    }
                    ++cnt;
                }
            }
        }
        if (cnt > KMAX) {
            atomicOr(&st->err, ERR_ROW);
            cnt = 0;
        }
    }
    uint32_t total;
    const uint32_t excl = block_excl_scan(cnt, s_w, total);
    s_excl[t] = excl;
    if (t == 0) {
        // the tile's own region of the contact list: no device-wide counter
        s_excl[TILE] = total;
        uint32_t base = tile * (uint32_t)TILE * slots;
        if (total > (uint32_t)TILE * slots) {
            atomicOr(&st->err, ERR_CAPACITY);
            atomicMax(&st->need, total);
            base = 0xFFFFFFFFu;
        } else {
            ts[tile].m += total;
        }
        s_base = base;
    }
    __syncthreads();
    const uint32_t base = s_base;
    if (base == 0xFFFFFFFFu) return;
    if (i < n) rows[i] = make_uint2(base + excl, cnt);
    for (uint32_t q = t; q < total; q += TILE) {
        const int o = owner_of(s_excl, q);
        col_j[base + q] = s_j[(q - s_excl[o]) * TILE + o];
    }
}

// ------------------------------------------------------------- contact law
// Eq. (2), (3), the stiffnesses and damping of section 2, Eq. (1), the
// sliding cap Eq. (4) with the displacement recomputed from the capped force,
// and the torque r_i (n x F).  R is the arithmetic type of the force (float
// in mixed precision, double in FP64); the tangential displacement is carried
// and updated in FP64.
template <typename R>
__device__ inline void contact_law(R nx, R ny, R nz, R dn, R vx, R vy, R vz, R rwx, R rwy,
                                   R rwz, double& dtx, double& dty, double& dtz, R rs, R ms, R ri,
                                   R kn_pref, R kt_pref, R alpha, R mu, double dt, R* F, R* T) {
    const R vns = vx * nx + vy * ny + vz * nz;
    const R vnx = vns * nx, vny = vns * ny, vnz = vns * nz;
    const R vtx = vx - vnx + (rwy * nz - rwz * ny);
    const R vty = vy - vny + (rwz * nx - rwx * nz);
    const R vtz = vz - vnz + (rwx * ny - rwy * nx);
    const double Nx = (double)nx, Ny = (double)ny, Nz = (double)nz;
    const double dtn = dtx * Nx + dty * Ny + dtz * Nz;
    dtx = dtx - dtn * Nx + (double)vtx * dt;
    dty = dty - dtn * Ny + (double)vty * dt;
    dtz = dtz - dtn * Nz + (double)vtz * dt;
    const R sdn = sqrt(dn);
    const R srs = sqrt(rs);
    const R kn = kn_pref * srs;
    const R kt = kt_pref * srs * sdn;
    const R eta = alpha * sqrt(ms * kn * sdn);
    const R el = kn * dn * sdn;
    const R Fnx = -el * nx - eta * vnx, Fny = -el * ny - eta * vny, Fnz = -el * nz - eta * vnz;
    R Ftx = -kt * (R)dtx - eta * vtx, Fty = -kt * (R)dty - eta * vty, Ftz = -kt * (R)dtz - eta * vtz;
    const R fn = sqrt(Fnx * Fnx + Fny * Fny + Fnz * Fnz);
    const R ft = sqrt(Ftx * Ftx + Fty * Fty + Ftz * Ftz);
    if (ft > mu * fn) {
        const R sc = mu * fn / ft;
        Ftx *= sc;
        Fty *= sc;
        Ftz *= sc;
        dtx = -(double)Ftx / (double)kt;
        dty = -(double)Fty / (double)kt;
        dtz = -(double)Ftz / (double)kt;
    }
    F[0] = Fnx + Ftx;
    F[1] = Fny + Fty;
    F[2] = Fnz + Ftz;
    T[0] = ri * (ny * F[2] - nz * F[1]);
    T[1] = ri * (nz * F[0] - nx * F[2]);
    T[2] = ri * (nx * F[1] - ny * F[0]);
}

// ------------------------------------------------------------------ force
template <typename R>
__global__ __launch_bounds__(TILE) void k_force(
    const double4* __restrict__ xr, const double2* __restrict__ vw, const uint8_t* __restrict__ mat,
    double4* __restrict__ xr_b, double2* __restrict__ vw_b, uint8_t* __restrict__ mat_b,
    const uint2* __restrict__ rows, const uint32_t* __restrict__ col_j,
    const uint2* __restrict__ rows_old, const uint32_t* __restrict__ prev,
    const uint32_t* __restrict__ tab_pid_old, const double* __restrict__ tab_dt_old,
    uint32_t* __restrict__ tab_pid_new, double* __restrict__ tab_dt_new, uint64_t cap,
    uint2* __restrict__ cells, uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
    R* __restrict__ fo, const MatTable* __restrict__ mt, uint32_t n, Geo G,
    TileStats* __restrict__ ts, Status* st) {
    __shared__ double4 s_x[TILE];
    __shared__ double2 s_vw[3][TILE];
    __shared__ uint2 s_old[TILE];
    __shared__ uint32_t s_excl[TILE + 1];
    __shared__ R s_f[6][TILE];
    __shared__ uint8_t s_mat[TILE];
    __shared__ uint32_t s_base, s_total, s_flag;
    __shared__ uint32_t s_red[4];
    if (skip_if_error(st, &s_flag)) return;

    const int t = threadIdx.x;
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t p0 = tile * TILE;
    const uint32_t i = p0 + t;
    const uint32_t nt = (n - p0) < (uint32_t)TILE ? (n - p0) : (uint32_t)TILE;
    uint2 row = make_uint2(0, 0);
    uint2 orow = make_uint2(0, 0);
    if (i < n) {
        row = rows[i];
        orow = rows_old[prev[i]];
        s_x[t] = xr[i];
        s_vw[0][t] = vw[i];
        s_vw[1][t] = vw[n + i];
        s_vw[2][t] = vw[2 * (size_t)n + i];
        s_mat[t] = mat ? mat[i] : (uint8_t)0;
    }
    s_old[t] = orow;
    if (t == 0) s_base = row.x;
    if ((uint32_t)t == nt - 1) s_total = row.x + row.y;
    __syncthreads();
    const uint32_t base = s_base;
    const uint32_t total = s_total - base;
    s_excl[t] = (i < n) ? row.x - base : total;
    if (t == 0) s_excl[TILE] = total;
    __syncthreads();
    if ((uint64_t)base + total > cap) {  // cannot happen after a clean detect
        if (t == 0) atomicOr(&st->err, ERR_CAPACITY);
        return;
    }

    R acc[6] = {0, 0, 0, 0, 0, 0};
    uint32_t matched = 0;
    const uint32_t my0 = s_excl[t], my1 = my0 + ((i < n) ? row.y : 0u);
    for (uint32_t c0 = 0; c0 < total; c0 += TILE) {
        const uint32_t q = c0 + t;
        if (q < total) {
            const int o = owner_of(s_excl, q);
            const uint32_t g = base + q;
            const uint32_t code = col_j[g];
            const double4 a = s_x[o];
            const double2 a0 = s_vw[0][o], a1 = s_vw[1][o], a2 = s_vw[2][o];
            const int mi = s_mat[o];
            const R ri = (R)meta_r(a.w);
            const double rid = (double)meta_r(a.w);
            const R mass_i = (R)(mt->mass_pref[mi] * rid * rid * rid);
            R nx, ny, nz, dn, vx, vy, vz, rwx, rwy, rwz, rs, ms;
            int mj;
            uint32_t pid_j;
            if (code < FACE) {
                const uint32_t j = code;
                const double4 b = xr[j];
                const double2 b0 = vw[j], b1 = vw[n + j], b2 = vw[2 * (size_t)n + j];
                mj = mat ? mat[j] : 0;
                pid_j = meta_pid(b.w);
                const double rjd = (double)meta_r(b.w);
                const R rj = (R)meta_r(b.w);
                double dx = b.x - a.x, dy = b.y - a.y, dz = b.z - a.z;
                int ky = 0;
                if (G.periodic) {
                    double Sx, Sy, Sz;
                    image_shift(G, dx, dy, dz, Sx, Sy, Sz, ky);
                    dx = dx + Sx;
                    dy = dy + Sy;
                    dz = dz + Sz;
                }
                const double d2 = dx * dx + dy * dy + dz * dz;
                const double s = rid + rjd;
                if (sizeof(R) == 8) {
                    const double d = sqrt(d2);
                    nx = (R)(dx / d);
                    ny = (R)(dy / d);
                    nz = (R)(dz / d);
                    dn = (R)(s - d);
                } else {
                    // overlap from (s^2 - d^2) / (s + d): the subtraction in FP64
                    // avoids the cancellation of s - d in FP32
                    const float d32 = sqrtf((float)d2);
                    const float inv = 1.0f / d32;
                    nx = (R)((float)dx * inv);
                    ny = (R)((float)dy * inv);
                    nz = (R)((float)dz * inv);
                    dn = (R)((float)(s * s - d2) / ((float)s + d32));
                }
                vx = (R)((a0.x - b0.x) - (double)ky * G.le_dv);
                vy = (R)(a0.y - b0.y);
                vz = (R)(a1.x - b1.x);
                rwx = ri * (R)a1.y + rj * (R)b1.y;
                rwy = ri * (R)a2.x + rj * (R)b2.x;
                rwz = ri * (R)a2.y + rj * (R)b2.y;
                rs = ri * rj / (ri + rj);
                const R mass_j = (R)(mt->mass_pref[mj] * rjd * rjd * rjd);
                ms = mass_i * mass_j / (mass_i + mass_j);
            } else {
                const int f = (int)(code - FACE), ax = f >> 1;
                pid_j = code;
                mj = mi;
                const double p = ax == 0 ? a.x : (ax == 1 ? a.y : a.z);
                const double dist = (f & 1) ? G.hi[ax] - p : p - G.lo[ax];
                const R sg = (f & 1) ? (R)1 : (R)-1;
                nx = ax == 0 ? sg : (R)0;
                ny = ax == 1 ? sg : (R)0;
                nz = ax == 2 ? sg : (R)0;
                dn = (R)(rid - dist);
                vx = (R)a0.x;
                vy = (R)a0.y;
                vz = (R)a1.x;
                rwx = ri * (R)a1.y;
                rwy = ri * (R)a2.x;
                rwz = ri * (R)a2.y;
                rs = ri;
                ms = mass_i;
            }
            // history: the previous step's row of this particle, sorted by partner id
            double dtx = 0.0, dty = 0.0, dtz = 0.0;
            const uint2 orw = s_old[o];
            for (uint32_t k = orw.x; k < orw.x + orw.y; ++k) {
                const uint32_t pk = tab_pid_old[k];
                if (pk == pid_j) {
                    dtx = tab_dt_old[k];
                    dty = tab_dt_old[(size_t)cap + k];
                    dtz = tab_dt_old[2 * (size_t)cap + k];
                    ++matched;
                    break;
                }
                if (pk > pid_j) break;
            }
            const int pr = mi * MAXMAT + mj;
            R F[3], T[3];
            contact_law<R>(nx, ny, nz, dn, vx, vy, vz, rwx, rwy, rwz, dtx, dty, dtz, rs, ms, ri,
                           (R)mt->kn_pref[pr], (R)mt->kt_pref[pr], (R)mt->alpha[pr],
                           (R)mt->mu[pr], G.dt, F, T);
            tab_pid_new[g] = pid_j;
            tab_dt_new[g] = dtx;
            tab_dt_new[(size_t)cap + g] = dty;
            tab_dt_new[2 * (size_t)cap + g] = dtz;
            s_f[0][t] = F[0];
            s_f[1][t] = F[1];
            s_f[2][t] = F[2];
            s_f[3][t] = T[0];
            s_f[4][t] = T[1];
            s_f[5][t] = T[2];
        }
        __syncthreads();
        // each particle adds its own contacts of this chunk in row order
        const uint32_t lo = my0 > c0 ? my0 : c0;
        const uint32_t hi = my1 < c0 + TILE ? my1 : c0 + TILE;
        for (uint32_t k = lo; k < hi; ++k) {
#pragma unroll
            for (int c = 0; c < 6; ++c) acc[c] += s_f[c][k - c0];
        }
        __syncthreads();
    }

    // churn counters into this tile's own slot
    {
        uint32_t mv = matched, ov = (i < n) ? orow.y : 0u;
        for (int o = 32; o > 0; o >>= 1) {
            mv += __shfl_down(mv, o, 64);
            ov += __shfl_down(ov, o, 64);
        }
        if ((t & 63) == 0) {
            s_red[2 * (t >> 6)] = mv;
            s_red[2 * (t >> 6) + 1] = ov;
        }
        __syncthreads();
        if (t == 0) {
            ts[tile].matched += s_red[0] + s_red[2];
            ts[tile].old += s_red[1] + s_red[3];
        }
    }
    if (i >= n) return;

    // per-particle totals, gravity, semi-implicit Euler (FP64)
    const double4 a = s_x[t];
    const double2 a0 = s_vw[0][t], a1 = s_vw[1][t], a2 = s_vw[2][t];
    const int mi = s_mat[t];
    const double r = (double)meta_r(a.w);
    const double m = mt->mass_pref[mi] * r * r * r;
    const double I = 0.4 * m * r * r;
    const double Fx = (double)acc[0] + m * G.g[0];
    const double Fy = (double)acc[1] + m * G.g[1];
    const double Fz = (double)acc[2] + m * G.g[2];
    double vx = a0.x + G.dt * Fx / m;
    double vy = a0.y + G.dt * Fy / m;
    double vz = a1.x + G.dt * Fz / m;
    double x = a.x + G.dt * vx;
    double y = a.y + G.dt * vy;
    double z = a.z + G.dt * vz;
    const double wx = a1.y + G.dt * (double)acc[3] / I;
    const double wy = a2.x + G.dt * (double)acc[4] / I;
    const double wz = a2.y + G.dt * (double)acc[5] / I;
    if (G.periodic & 2u) {
        if (y >= G.hi[1]) {
            y -= G.L[1];
            x -= G.le_shift_next;
            vx -= G.le_dv;
        } else if (y < G.lo[1]) {
            y += G.L[1];
            x += G.le_shift_next;
            vx += G.le_dv;
        }
    }
    // bounded wraps: a non-finite coordinate stays non-finite and is flagged
    if (G.periodic & 1u) {
        for (int k = 0; k < 4 && x >= G.hi[0]; ++k) x -= G.L[0];
        for (int k = 0; k < 4 && x < G.lo[0]; ++k) x += G.L[0];
    }
    if (G.periodic & 4u) {
        for (int k = 0; k < 4 && z >= G.hi[2]; ++k) z -= G.L[2];
        for (int k = 0; k < 4 && z < G.lo[2]; ++k) z += G.L[2];
    }
    const bool finite = isfinite(x) && isfinite(y) && isfinite(z) && isfinite(vx) &&
                        isfinite(vy) && isfinite(vz) && isfinite(wx) && isfinite(wy) &&
                        isfinite(wz);
    if (!finite) atomicOr(&st->err, ERR_NONFINITE);
    xr_b[i] = make_double4(x, y, z, a.w);
    vw_b[i] = make_double2(vx, vy);
    vw_b[n + i] = make_double2(vz, wx);
    vw_b[2 * (size_t)n + i] = make_double2(wy, wz);
    if (mat_b) mat_b[i] = (uint8_t)mi;
    keys[i] = cell_key(G, x, y, z);
    vals[i] = i;
    if (fo) {
        fo[i] = (R)Fx;
        fo[n + i] = (R)Fy;
        fo[2 * (size_t)n + i] = (R)Fz;
        fo[3 * (size_t)n + i] = acc[3];
        fo[4 * (size_t)n + i] = acc[4];
        fo[5 * (size_t)n + i] = acc[5];
    }
    // the first particle of its (old) cell empties the cell's bounds; the
    // reorder kernel writes the bounds of the new order
    const uint32_t lin = key_lin(G, cell_key(G, a.x, a.y, a.z));
    if (cells[lin].x == i) cells[lin] = make_uint2(0, 0);
}

// ------------------------------------------------------------------ hash
__global__ void k_hash(const double4* __restrict__ xr, uint32_t n, Geo G, uint32_t* keys,
                       uint32_t* vals) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double4 a = xr[i];
    keys[i] = cell_key(G, a.x, a.y, a.z);
    vals[i] = i;
}

// ------------------------------------------------------------- radix sort
// Pass over one 8-bit digit: per-tile digit histograms, a scan of the
// (digit, tile) counts, then a stable scatter.
__global__ __launch_bounds__(SORT_THREADS) void k_radix_hist(const uint32_t* __restrict__ keys,
                                                             uint32_t n, int shift,
                                                             uint32_t* __restrict__ tile_hist,
                                                             uint32_t ntiles, const Status* st) {
    __shared__ uint32_t h[256];
    __shared__ uint32_t s_flag;
    if (skip_if_error(st, &s_flag)) return;
    const int t = threadIdx.x;
    h[t] = 0;
    __syncthreads();
    const uint32_t b = blockIdx.x * SORT_TILE;
#pragma unroll
    for (int q = 0; q < SORT_ITEMS; ++q) {
        const uint32_t idx = b + q * SORT_THREADS + t;
        if (idx < n) atomicAdd(&h[(keys[idx] >> shift) & 255u], 1u);
    }
    __syncthreads();
    tile_hist[t * ntiles + blockIdx.x] = h[t];
}

__device__ inline uint32_t block256_excl_scan(uint32_t v, uint32_t* s_w, uint32_t& total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t u = __shfl_up(x, o, 64);
        if (lane >= o) x += u;
    }
    if (lane == 63) s_w[w] = x;
    __syncthreads();
    uint32_t off = 0;
    for (int k = 0; k < w; ++k) off += s_w[k];
    total = s_w[0] + s_w[1] + s_w[2] + s_w[3];
    __syncthreads();
    return x - v + off;
}

// One workgroup per digit: exclusive scan of that digit's per-tile counts.
__global__ __launch_bounds__(SORT_THREADS) void k_radix_scan(uint32_t* __restrict__ tile_hist,
                                                             uint32_t ntiles,
                                                             uint32_t* __restrict__ digit_tot,
                                                             const Status* st) {
    __shared__ uint32_t s_w[4];
    __shared__ uint32_t s_flag;
    if (skip_if_error(st, &s_flag)) return;
    uint32_t* row = tile_hist + (size_t)blockIdx.x * ntiles;
    uint32_t carry = 0;
    for (uint32_t c0 = 0; c0 < ntiles; c0 += SORT_THREADS) {
        const uint32_t k = c0 + threadIdx.x;
        const uint32_t v = k < ntiles ? row[k] : 0u;
        uint32_t tot;
        const uint32_t e = block256_excl_scan(v, s_w, tot);
        if (k < ntiles) row[k] = carry + e;
        carry += tot;
    }
    if (threadIdx.x == 0) digit_tot[blockIdx.x] = carry;
}

__global__ __launch_bounds__(SORT_THREADS) void k_radix_scatter(
    const uint32_t* __restrict__ keys_in, const uint32_t* __restrict__ vals_in,
    uint32_t* __restrict__ keys_out, uint32_t* __restrict__ vals_out, uint32_t n, int shift,
    const uint32_t* __restrict__ tile_hist, const uint32_t* __restrict__ digit_tot, uint32_t ntiles,
    const Status* st) {
    __shared__ uint32_t s_base[256];   // global offset of each digit for this tile
    __shared__ uint32_t s_run[256];    // keys of each digit already placed by this tile
    __shared__ uint32_t s_wc[4][256];  // per-wave digit counts, then per-wave offsets
    __shared__ uint32_t s_w[4];
    __shared__ uint32_t s_flag;
    if (skip_if_error(st, &s_flag)) return;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    {
        uint32_t tot;
        const uint32_t e = block256_excl_scan(digit_tot[t], s_w, tot);
        s_base[t] = e + tile_hist[t * ntiles + blockIdx.x];
        s_run[t] = 0;
    }
    const unsigned long long lt = (1ull << lane) - 1ull;
    const uint32_t b = blockIdx.x * SORT_TILE;
    for (int q = 0; q < SORT_ITEMS; ++q) {
        const uint32_t idx = b + q * SORT_THREADS + t;
        const bool valid = idx < n;
        const uint32_t key = valid ? keys_in[idx] : 0u;
        const uint32_t val = valid ? vals_in[idx] : 0u;
        const uint32_t d = (key >> shift) & 255u;
        // lanes of this wave holding the same digit
        unsigned long long peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool on = (d >> bit) & 1u;
            const unsigned long long bal = __ballot(on);
            peers &= on ? bal : ~bal;
        }
        s_wc[0][t] = 0;
        s_wc[1][t] = 0;
        s_wc[2][t] = 0;
        s_wc[3][t] = 0;
        __syncthreads();
        const uint32_t rank = (uint32_t)__popcll(peers & lt);
        if (valid && rank == 0) s_wc[w][d] = (uint32_t)__popcll(peers);
        __syncthreads();
        {
            // thread t owns digit t: turn per-wave counts into offsets
            uint32_t run = s_run[t];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const uint32_t c = s_wc[k][t];
                s_wc[k][t] = run;
                run += c;
            }
            s_run[t] = run;
        }
        __syncthreads();
        if (valid) {
            const uint32_t dst = s_base[d] + s_wc[w][d] + rank;
            keys_out[dst] = key;
            vals_out[dst] = val;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ reorder
__global__ void k_reorder(const uint32_t* __restrict__ keys_s, const uint32_t* __restrict__ vals_s,
                          const double4* __restrict__ xr_b, const double2* __restrict__ vw_b,
                          const uint8_t* __restrict__ mat_b, double4* __restrict__ xr,
                          double2* __restrict__ vw, uint8_t* __restrict__ mat,
                          uint32_t* __restrict__ prev, uint2* __restrict__ cells, uint32_t n, Geo G,
                          Status* st, int count_step) {
    __shared__ uint32_t s_flag;
    if (skip_if_error(st, &s_flag)) return;
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && count_step) st->steps_done += 1;
    if (i >= n) return;
    const uint32_t src = vals_s[i];
    xr[i] = xr_b[src];
    vw[i] = vw_b[src];
    vw[n + i] = vw_b[n + src];
    vw[2 * (size_t)n + i] = vw_b[2 * (size_t)n + src];
    if (mat) mat[i] = mat_b[src];
    prev[i] = src;
    const uint32_t key = keys_s[i];
    const uint32_t lin = key_lin(G, key);
    if (i == 0 || keys_s[i - 1] != key) cells[lin].x = i;
    if (i == n - 1 || keys_s[i + 1] != key) cells[lin].y = i + 1;
}

// ------------------------------------------------------------------ launch
void launch_detect(int kmax, const State& A, const uint2* cells, uint32_t n, const Geo& G,
                   uint2* rows, uint32_t* col_j, uint32_t slots, TileStats* ts, Status* st,
                   hipStream_t s) {
    if (n == 0) return;
    const uint32_t nb = (n + TILE - 1) / TILE;
    if (kmax <= 16)
        hipLaunchKernelGGL(k_detect<16>, dim3(nb), dim3(TILE), 0, s, A.xr, cells, n, G, rows,
                           col_j, slots, ts, st);
    else
        hipLaunchKernelGGL(k_detect<64>, dim3(nb), dim3(TILE), 0, s, A.xr, cells, n, G, rows,
                           col_j, slots, ts, st);
}

void launch_force(bool fp64, const State& A, const State& B, const uint2* rows,
                  const uint32_t* col_j, const uint2* rows_old, const uint32_t* prev,
                  const uint32_t* tab_pid_old, const double* tab_dt_old, uint32_t* tab_pid_new,
                  double* tab_dt_new, uint64_t cap, uint2* cells, uint32_t* keys, uint32_t* vals,
                  void* fo, const MatTable* mt, uint32_t n, const Geo& G, TileStats* ts,
                  Status* st, hipStream_t s) {
    if (n == 0) return;
    const uint32_t nb = (n + TILE - 1) / TILE;
    if (fp64)
        hipLaunchKernelGGL(k_force<double>, dim3(nb), dim3(TILE), 0, s, A.xr, A.vw, A.mat, B.xr,
                           B.vw, B.mat, rows, col_j, rows_old, prev, tab_pid_old, tab_dt_old,
                           tab_pid_new, tab_dt_new, cap, cells, keys, vals, (double*)fo, mt, n, G,
                           ts, st);
    else
        hipLaunchKernelGGL(k_force<float>, dim3(nb), dim3(TILE), 0, s, A.xr, A.vw, A.mat, B.xr,
                           B.vw, B.mat, rows, col_j, rows_old, prev, tab_pid_old, tab_dt_old,
                           tab_pid_new, tab_dt_new, cap, cells, keys, vals, (float*)fo, mt, n, G,
                           ts, st);
}

void launch_hash(const State& B, uint32_t n, const Geo& G, uint32_t* keys, uint32_t* vals,
                 hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_hash, dim3((n + 255) / 256), dim3(256), 0, s, B.xr, n, G, keys, vals);
}

size_t sort_hist_words(uint32_t n) {
    const size_t ntiles = (n + SORT_TILE - 1) / SORT_TILE;
    return 256 * (ntiles ? ntiles : 1) + 256;
}

void launch_radix_sort(uint32_t* keys, uint32_t* vals, uint32_t* keys_tmp, uint32_t* vals_tmp,
                       uint32_t n, int bits, uint32_t* tile_hist, uint32_t* digit_tot,
                       uint32_t** keys_out, uint32_t** vals_out, const Status* st, hipStream_t s) {
    uint32_t *ki = keys, *vi = vals, *ko = keys_tmp, *vo = vals_tmp;
    if (n > 1) {
        const uint32_t ntiles = (n + SORT_TILE - 1) / SORT_TILE;
        for (int shift = 0; shift < bits; shift += 8) {
            hipLaunchKernelGGL(k_radix_hist, dim3(ntiles), dim3(SORT_THREADS), 0, s, ki, n, shift,
                               tile_hist, ntiles, st);
            hipLaunchKernelGGL(k_radix_scan, dim3(256), dim3(SORT_THREADS), 0, s, tile_hist, ntiles,
                               digit_tot, st);
            hipLaunchKernelGGL(k_radix_scatter, dim3(ntiles), dim3(SORT_THREADS), 0, s, ki, vi, ko,
                               vo, n, shift, tile_hist, digit_tot, ntiles, st);
            uint32_t* tk = ki;
            ki = ko;
            ko = tk;
            uint32_t* tv = vi;
            vi = vo;
            vo = tv;
        }
    }
    *keys_out = ki;
    *vals_out = vi;
}

void launch_reorder(const uint32_t* keys_s, const uint32_t* vals_s, const State& B, const State& A,
                    uint32_t* prev, uint2* cells, uint32_t n, const Geo& G, Status* st,
                    int count_step, hipStream_t s) {
    const uint32_t nb = n ? (n + 255) / 256 : 1;
    hipLaunchKernelGGL(k_reorder, dim3(nb), dim3(256), 0, s, keys_s, vals_s, B.xr, B.vw, B.mat,
                       A.xr, A.vw, A.mat, prev, cells, n, G, st, count_step);
}

}  // namespace dem
