// HIP kernels of one DEM step for CDNA4 (gfx950, wave64).
//
// Step = contact search -> force -> sort -> reorder, all on one stream:
//
//  search   the paper's first loop (section 3.4: collect the ids of touching
//           partners first).  Default (k_detect_half): one lane per particle
//           scans the upper half of the 27-cell stencil around it (section
//           3.3, "cell-based method"), so each pair is tested once, and
//           enters every contact in both particles' adjacency lists.  With
//           DEM_FLAG_FULL_DETECT (k_detect): the lane scans all 27 cells and
//           keeps its partners in an LDS row ordered by partner id; the
//           workgroup compacts its 128 rows into its own region of the
//           contact list.
//  force    the second loop: the workgroup first turns its particles' lists
//           into rows ordered by partner id (default path), then runs one
//           lane per compacted contact: history match against the previous
//           step's table, the contact law (Eq. 1-4, torque), a per-particle
//           sum in ascending partner id through LDS, gravity
//           ("ForceGravity"), semi-implicit Euler ("Integrate"), and the new
//           cell key ("CalcHash").  Every lane of a wavefront is busy on a
//           real contact.
//  sort     the particles that changed cell are merged into the unchanged
//           ones ("BitonicSort" in the paper); an LSD radix sort (8-bit
//           digits, wave64 ballot ranking) is the fallback.
//  reorder  the permutation into the new cell order, the gathered position
//           records and the cell bounds ("FindCellBoundsAndReorder").
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>

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

// Cell key: Morton (bit-interleaved) order over the (y, z) rows of cells,
// with the x index as the fastest-varying part.  Rows that are close in
// (y, z) stay close in memory, and the three x-neighbouring cells of a row
// are consecutive keys, so their particles form one contiguous range.
__device__ inline uint32_t spread2(uint32_t v) {
    v &= 0xFFFFu;
    v = (v | (v << 8)) & 0x00FF00FFu;
    v = (v | (v << 4)) & 0x0F0F0F0Fu;
    v = (v | (v << 2)) & 0x33333333u;
    v = (v | (v << 1)) & 0x55555555u;
    return v;
}
__device__ inline uint32_t compact2(uint32_t v) {
    v &= 0x55555555u;
    v = (v ^ (v >> 1)) & 0x33333333u;
    v = (v ^ (v >> 2)) & 0x0F0F0F0Fu;
    v = (v ^ (v >> 4)) & 0x00FF00FFu;
    v = (v ^ (v >> 8)) & 0x0000FFFFu;
    return v;
}
__device__ inline uint32_t cell_key(const Geo& G, double x, double y, double z) {
    const uint32_t cx = (uint32_t)cell_coord(G, x, 0), cy = (uint32_t)cell_coord(G, y, 1),
                   cz = (uint32_t)cell_coord(G, z, 2);
    return ((spread2(cy) | (spread2(cz) << 1)) << G.xbits) | cx;
}
__device__ inline uint32_t key_lin(const Geo& G, uint32_t key) {
    const uint32_t cx = key & ((1u << G.xbits) - 1u), m = key >> G.xbits;
    const uint32_t cy = compact2(m), cz = compact2(m >> 1);
    return (cz * (uint32_t)G.nc[1] + cy) * (uint32_t)G.nc[0] + cx;
}

// Image of partner j that can touch i: periodic copies by minimum image, the
// Lees-Edwards copy across y carrying the shear offset along x.  Returns the
// shift S added to the raw difference x_j - x_i and the y-image index.  For a
// touching pair |d + k L| < L / 3, so rounding d / L (here d times 1 / L) to
// the nearest integer picks the same image however it is rounded.
__device__ inline void image_shift(const Geo& G, double dx, double dy, double dz, double& Sx,
                                   double& Sy, double& Sz, int& ky) {
    ky = 0;
    Sx = Sy = Sz = 0.0;
    if (G.periodic & 2u) {
        ky = -(int)rint(dy * G.inv_L[1]);
        Sy = (double)ky * G.L[1];
    }
    if (G.periodic & 1u) {
        double dxp = dx + (double)ky * G.le_shift;
        int kx = -(int)rint(dxp * G.inv_L[0]);
        Sx = (double)kx * G.L[0] + (double)ky * G.le_shift;
    }
    if (G.periodic & 4u) {
        int kz = -(int)rint(dz * G.inv_L[2]);
        Sz = (double)kz * G.L[2];
    }
}

// The FP32 record of the contact search: position relative to the box corner
// and radius.  Within 3 box lengths of the corner the float rounding error is
// bounded (see detect_margin); a particle further out gets NaN coordinates,
// which make every pre-filter comparison involving it pass.
__device__ inline float4 far_record(const Geo& G, const double4& p) {
    const double rx = p.x - G.lo[0], ry = p.y - G.lo[1], rz = p.z - G.lo[2];
    const bool near = fabs(rx) <= 3.0 * G.L[0] && fabs(ry) <= 3.0 * G.L[1] && fabs(rz) <= 3.0 * G.L[2];
    const float q = __int_as_float(0x7fc00000);
    return near ? make_float4((float)rx, (float)ry, (float)rz, meta_r(p.w))
                : make_float4(q, q, q, meta_r(p.w));
}

// Squared centre distance ((dx^2 + dy^2) + dz^2) with no fused multiply-add:
// the contact predicate and the contact geometry both use it, so a pair the
// predicate accepts has d2 < s^2 in the force computation as well.
__device__ inline double dist2(double dx, double dy, double dz) {
#pragma clang fp contract(off)
    double d2 = dx * dx + dy * dy;
    d2 = d2 + dz * dz;
    return d2;
}

// The contact predicate on FP64 positions, written out with no fused
// multiply-add so that the contact set is bit-exact: ((dx^2+dy^2)+dz^2) < s^2.
__device__ inline bool touching(double dx, double dy, double dz, double s) {
#pragma clang fp contract(off)
    return dist2(dx, dy, dz) < s * s;
}

// Extra wall W and a centre c: w = q - c for the wall's point q closest to c
// (the rectangle's or segment's parameters clamped to [0, 1]); returns
// |w|^2.  Written out with no fused multiply-add, so that the contact
// decision |w|^2 < r^2 is bit-exact.
__device__ inline double wall_gap(const dem_wall& W, double cx, double cy, double cz, double& wx,
                                  double& wy, double& wz) {
#pragma clang fp contract(off)
    const double dx = cx - W.p[0], dy = cy - W.p[1], dz = cz - W.p[2];
    double s = (dx * W.u[0] + dy * W.u[1] + dz * W.u[2]) /
               (W.u[0] * W.u[0] + W.u[1] * W.u[1] + W.u[2] * W.u[2]);
    s = s < 0.0 ? 0.0 : (s > 1.0 ? 1.0 : s);
    double qx = W.p[0] + s * W.u[0], qy = W.p[1] + s * W.u[1], qz = W.p[2] + s * W.u[2];
    if (W.kind == DEM_WALL_RECT) {
        double t = (dx * W.v[0] + dy * W.v[1] + dz * W.v[2]) /
                   (W.v[0] * W.v[0] + W.v[1] * W.v[1] + W.v[2] * W.v[2]);
        t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
        qx = qx + t * W.v[0];
        qy = qy + t * W.v[1];
        qz = qz + t * W.v[2];
    }
    wx = qx - cx;
    wy = qy - cy;
    wz = qz - cz;
    const double d2 = wx * wx + wy * wy;
    return d2 + wz * wz;
}

// Whether a sphere of radius r centred at c touches extra wall W (a centre
// exactly on a segment makes no contact).
__device__ inline bool wall_touch(const dem_wall& W, double cx, double cy, double cz, double r) {
    double wx, wy, wz;
    const double d2 = wall_gap(W, cx, cy, cz, wx, wy, wz);
    return d2 < r * r && (W.kind == DEM_WALL_RECT || d2 > 0.0);
}

// Data that no kernel writes while it reads them (the job descriptors, the
// tile maps) and the error word of the step, at workgroup-uniform addresses,
// are read through the constant address space: scalar loads into SGPRs,
// which wait on no vector load issued before them and take no vector
// registers.  The scalar cache is invalidated at every kernel launch, so such
// a load sees what earlier kernels of the stream wrote.
template <typename T>
using ConstPtr = const __attribute__((address_space(4))) T*;

// Whether an earlier kernel of the step (or, at times, another workgroup of
// this one) reported an error; the same answer for the whole workgroup.
__device__ inline uint32_t skip_if_error(const Status* st, uint32_t* s_flag) {
    const uint32_t e = ((ConstPtr<Status>)st)->err;
    if (threadIdx.x == 0) *s_flag = e;
    __syncthreads();
    return *s_flag;
}

// The running job of a tile, or null for a free tile or a job that is
// finished or failed.  The descriptor is read at a workgroup-uniform address
// through the constant address space, so its fields come in through scalar
// loads and stay in SGPRs.
__device__ inline const Job* tile_job(const Job* __restrict__ jobs, const PoolView& P,
                                      uint32_t tile, uint32_t& jb) {
    jb = ((ConstPtr<uint32_t>)P.tile_job)[tile];
    if (jb == NO_JOB) return nullptr;
    ConstPtr<Job> J = (ConstPtr<Job>)jobs + jb;
    return J->status == JOB_ACTIVE ? (const Job*)J : nullptr;
}

// The key bits of a tile's segment (a job's tiles sort together).
__device__ inline uint32_t tile_key_of(const PoolView& P, uint32_t tile) {
    return ((ConstPtr<uint32_t>)P.tile_key)[tile];
}

// Exclusive scan of v over a workgroup of NW waves.
template <int NW>
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
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        off += (k < w) ? s_w[k] : 0u;
        tot += s_w[k];
    }
    total = tot;
    return x - v + off;
}

// Largest o in [0, NT) with e[o] <= q, for e non-decreasing with e[0] = 0.
template <int NT = TILE>
__device__ inline int owner_of(const uint32_t* e, uint32_t q) {
    int lo = 0, hi = NT;
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (e[mid] <= q) lo = mid;
        else hi = mid;
    }
    return lo;
}

// ------------------------------------------------------------------ detect
// Particles [lo, hi) of the non-empty cells among up to three consecutive
// cells of a row (consecutive keys, hence one contiguous range).
__device__ inline void merge_range(uint2 c, uint32_t& lo, uint32_t& hi) {
    if (c.y > c.x) {
        lo = c.x < lo ? c.x : lo;
        hi = c.y > hi ? c.y : hi;
    }
}

// Candidate ranges of the particle at a (radius ri), written to col[k * stride]
// (the lane's column of a range table); returns their number and, with
// `count`, adds up their lengths there.  The lane scans the 27 cells around
// the particle as 9 contiguous ranges: in each (y, z) row the three
// x-neighbouring cells are consecutive cell keys (plus, across a periodic x
// boundary, one wrapped cell).  All 27 cell bounds are loaded before any is
// used.
//
// HALF: only the upper half of the stencil, so that a pair of cells is
// scanned from one of its two cells: the rows one cell up in z, the row one
// cell up in y in the particle's own z layer, and in its own row the cell one
// up in x and the positions of its own cell above `self` (the particle's own
// position).  Cell offsets between two particles are exact negatives of each
// other, so every pair of particles in neighbouring cells is scanned from
// exactly one of its two particles.
template <bool PER, bool HALF = false>
__device__ __forceinline__ uint32_t candidate_ranges(const Geo& G, const double4& a, double ri,
                                                     const uint2* __restrict__ cells,
                                                     uint2* col, int stride,
                                                     uint32_t* count = nullptr,
                                                     uint32_t self = 0) {
    const int nx = G.nc[0], ny = G.nc[1], nz = G.nc[2];
    // without periodic jobs in the pool the wrap and shear code compiles away
    const bool px = PER && (G.periodic & 1u), py = PER && (G.periodic & 2u),
               pz = PER && (G.periodic & 4u), le = PER && G.le;
    uint32_t nw = 0;
    const int cx = cell_coord(G, a.x, 0), cy = cell_coord(G, a.y, 1), cz = cell_coord(G, a.z, 2);
    // Reach pruning: a partner lies within r_i + reach of the particle, so
    // a row of cells whose (y, z) slab is farther holds none, nor does an
    // x-neighbour cell beyond the reach left in x.  Per offset -1, 0, +1
    // along y and z: whether the neighbour row exists, its (wrapped)
    // index, and the squared gap from the particle to its slab.
    const double reach = ri + G.reach;
    const double reach2 = reach * reach;
    int qy[3], qz[3], ky[3];
    bool oky[3], okz[3];
    double gy2[3], gz2[3];
#pragma unroll
    for (int o = 0; o < 3; ++o) {
        const int d = o - 1;
        int y = cy + d, z = cz + d, kk = 0;
        bool ok_y = true, ok_z = true;
        if (y < 0 || y >= ny) {
            if (!py) ok_y = false;
            kk = y < 0 ? -1 : 1;
            y -= kk * ny;
        }
        if (z < 0 || z >= nz) {
            if (!pz) ok_z = false;
            z = z < 0 ? z + nz : z - nz;
        }
        qy[o] = y;
        qz[o] = z;
        ky[o] = kk;
        oky[o] = ok_y;
        okz[o] = ok_z;
        double g = 0.0, h = 0.0;
        if (d > 0) {
            g = fmax(0.0, G.lo[1] + (double)(cy + 1) * G.cw[1] - a.y);
            h = fmax(0.0, G.lo[2] + (double)(cz + 1) * G.cw[2] - a.z);
        } else if (d < 0) {
            g = fmax(0.0, a.y - (G.lo[1] + (double)cy * G.cw[1]));
            h = fmax(0.0, a.z - (G.lo[2] + (double)cz * G.cw[2]));
        }
        gy2[o] = g * g;
        gz2[o] = h * h;
    }
    const double dl = a.x - (G.lo[0] + (double)cx * G.cw[0]);
    const double dh = G.lo[0] + (double)(cx + 1) * G.cw[0] - a.x;
    const double dl2 = dl > 0.0 ? dl * dl : 0.0, dh2 = dh > 0.0 ? dh * dh : 0.0;

    // the 9 rows' three cells (main range, plus the wrapped x neighbour
    // with a periodic x axis); all 27 cell bounds are loaded before any is
    // used
    uint32_t il[9], im[9], ih[9];
    bool okl[9], okm[9], okh[9], wrl[9], wrh[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const int oz = k / 3, oy = k % 3;
        const double rx2 = reach2 - gy2[oy] - gz2[oz];
        const bool upper = oz == 2 || (oz == 1 && oy == 2);
        const bool own = oz == 1 && oy == 1;
        const bool ok = oky[oy] && okz[oz] && rx2 > 0.0 && (!HALF || upper || own);
        int cxq = cx;
        bool xprune = true;
        if (le && ky[oy] != 0) {
            // across a sheared y boundary the partner row is offset along x
            double fx = floor((a.x - (double)ky[oy] * G.le_shift - G.lo[0]) * G.inv_cell[0]);
            const double lim = 2.0 * (double)nx;
            if (!(fx >= -lim)) fx = -lim;  // also NaN
            if (fx > lim) fx = lim;
            cxq = (int)fx % nx;
            if (cxq < 0) cxq += nx;
            xprune = false;
        }
        int xl = cxq - 1, xh = cxq + 1;
        okm[k] = ok;
        okl[k] = ok && !(xprune && dl2 >= rx2) && !(HALF && own);
        okh[k] = ok && !(xprune && dh2 >= rx2);
        wrl[k] = wrh[k] = false;
        if (xl < 0) {
            if (px) { xl += nx; wrl[k] = true; } else okl[k] = false;
        }
        if (xh >= nx) {
            if (px) { xh -= nx; wrh[k] = true; } else okh[k] = false;
        }
        const uint32_t row = ok ? ((uint32_t)qz[oz] * (uint32_t)ny + (uint32_t)qy[oy]) * (uint32_t)nx : 0u;
        il[k] = okl[k] ? row + (uint32_t)xl : 0u;
        im[k] = ok ? row + (uint32_t)cxq : 0u;
        ih[k] = okh[k] ? row + (uint32_t)xh : 0u;
    }
    uint2 cl[9], cm[9], cr[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        cl[k] = cells[il[k]];
        cm[k] = cells[im[k]];
        cr[k] = cells[ih[k]];
    }
    // non-empty ranges to LDS, so one flat loop walks all candidates
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const uint2 z = make_uint2(0, 0);
        const uint2 l = okl[k] ? cl[k] : z, m = okm[k] ? cm[k] : z, h = okh[k] ? cr[k] : z;
        uint32_t lo = 0xFFFFFFFFu, hi = 0u, lo2 = 0xFFFFFFFFu, hi2 = 0u;
        merge_range(m, lo, hi);
        if (wrl[k]) merge_range(l, lo2, hi2); else merge_range(l, lo, hi);
        if (wrh[k]) merge_range(h, lo2, hi2); else merge_range(h, lo, hi);
        // own row of the half stencil: the own cell and, consecutive after
        // it, the unwrapped cell up in x; the wrapped one is in lo2..hi2
        if (HALF && k == 4) lo = lo < self + 1 ? self + 1 : lo;
        if (hi > lo) {
            col[(nw++) * stride] = make_uint2(lo, hi);
            if (count) *count += hi - lo;
        }
        if (PER && hi2 > lo2) {
            col[(nw++) * stride] = make_uint2(lo2, hi2);
            if (count) *count += hi2 - lo2;
        }
    }
    return nw;
}

// FP32 pre-filter of a candidate record: never rejects a pair that touches in
// FP64 (NaN records of particles far from the box always pass).
// CUT: a two-level job's walk, which leaves candidates above the radius cut
// to the wide scan.
template <bool PER, bool CUT = true>
struct PreFilter {
    float4 me;
    float Lx, Ly, Lz, Df, iLx, iLy, iLz, rm;
    float rc;  // candidates with a larger radius are the wide scan's (two-level search)
    uint32_t per;
    __device__ PreFilter(const Geo& G, const double4& a, float margin) {
        me = far_record(G, a);
        Lx = (float)G.L[0];
        Ly = (float)G.L[1];
        Lz = (float)G.L[2];
        Df = (float)G.le_shift;
        iLx = (float)G.inv_L[0];
        iLy = (float)G.inv_L[1];
        iLz = (float)G.inv_L[2];
        rm = me.w + margin;
        per = G.periodic;
        rc = G.rcut;
    }
    __device__ bool operator()(const float4& b) const {
        float dx = b.x - me.x, dy = b.y - me.y, dz = b.z - me.z;
        if (PER) {
            int ky = 0;
            if (per & 2u) {
                ky = -(int)rintf(dy * iLy);
                dy += (float)ky * Ly;
            }
            if (per & 1u) {
                const int kx = -(int)rintf((dx + (float)ky * Df) * iLx);
                dx += (float)kx * Lx + (float)ky * Df;
            }
            if (per & 4u) dz += (float)(-(int)rintf(dz * iLz)) * Lz;
        }
        const float sm = rm + b.w;
        return !(dx * dx + dy * dy + dz * dz >= sm * sm) && (!CUT || b.w <= rc);
    }
};

// The position record (FP64 position, radius and id) of a sorted position:
// the record in the state buffer the step reads, through the permutation.
// The sorted order keeps only the contact search's FP32 records; the FP64
// records are read where they are.
// A permutation entry is read for any position a lane may load, also ghost
// slots and free tiles, whose entries no step writes: an entry outside the
// arrays is taken as the position itself, so every load stays in bounds.
struct SortedPos {
    const double4* __restrict__ xr;   // the state buffer the step reads
    const uint32_t* __restrict__ perm;  // sorted position -> position in it
    uint32_t n;                         // positions in both arrays
    __device__ __forceinline__ double4 operator[](uint32_t j) const {
        const uint32_t q = perm[j];
        return xr[q < n ? q : j];
    }
};

// Exact FP64 re-walk of a lane's `nw` candidate ranges (win(k) gives range
// k) into its column of s_j; returns the number of contacts found.
template <int KMAX, bool PER, typename Win>
__device__ __forceinline__ uint32_t rewalk_exact(const PoolView& P, const Geo& G, const double4& a,
                                                 double ri, uint32_t i, int t, uint32_t nw,
                                                 Win win, SortedPos xr, uint32_t* s_j) {
    // more survivors than the row holds (a particle far from the box, whose
    // FP32 record passes every comparison, or a tight clump): walk the
    // candidates again with the exact FP64 test, so only more real contacts
    // than the row holds are an error
    uint32_t sc = 0;
    for (uint32_t w2 = 0; w2 < nw; ++w2) {
        const uint2 rg2 = win(w2);
        for (uint32_t jx = rg2.x; jx < rg2.y; ++jx) {
            if (jx == i || jx >= P.ns) continue;
            const double4 b = xr[jx];
            double dx = b.x - a.x, dy = b.y - a.y, dz = b.z - a.z;
            if (PER) {
                double Sx, Sy, Sz;
                int ky;
                image_shift(G, dx, dy, dz, Sx, Sy, Sz, ky);
                dx = dx + Sx;
                dy = dy + Sy;
                dz = dz + Sz;
            }
            if (touching(dx, dy, dz, ri + (double)meta_r(b.w))) {
                s_j[min(sc, (uint32_t)KMAX) * DTILE + t] = jx;
                ++sc;
            }
        }
    }
    return sc;
}

// The end of one lane's contact search, after pass 1 left `sc` survivors in
// its column of s_j: an exact re-walk of its `nw` candidate ranges (win(k)
// gives range k) when the survivors overflow the row, the exact FP64 test of the survivors with
// insertion by partner id, then the box faces.  Returns the row length (0
// after reporting a row overflow).  The partner ids live in the .x half of
// the lane's column pcol[k * pstride] of a range table.
template <int KMAX, bool PER, typename Win>
__device__ __forceinline__ uint32_t detect_row(const PoolView& P, const Geo& G, const double4& a,
                                               double ri, uint32_t i, int t, uint32_t sc,
                                               uint32_t nw, Win win, SortedPos xr, uint32_t* s_j,
                                               uint2* pcol, int pstride,
                                               const dem_wall* __restrict__ xw, uint32_t nxw) {
    auto pid_at = [&](int k) -> uint32_t& { return pcol[k * pstride].x; };
    uint32_t cnt = 0;
    if (sc > KMAX) sc = rewalk_exact<KMAX, PER>(P, G, a, ri, i, t, nw, win, xr, s_j);
    if (sc > KMAX) {
        cnt = KMAX + 1;  // row buffer too small: reported below
    } else {
        // pass 2: exact FP64 test of the survivors, four loads in flight;
        // a hit goes into the row in partner-id order (a group's partner
        // indices are read before any insertion, and insertion only
        // writes slots up to the hit count)
        for (uint32_t q0 = 0; q0 < sc; q0 += 4) {
            uint32_t jj[4];
            double4 bb[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) jj[m] = q0 + m < sc ? s_j[(q0 + m) * DTILE + t] : 0xFFFFFFFFu;
#pragma unroll
            for (int m = 0; m < 4; ++m) bb[m] = xr[jj[m] < P.ns ? jj[m] : i];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                if (jj[m] == 0xFFFFFFFFu) continue;
                const double4 b = bb[m];
                double dx = b.x - a.x, dy = b.y - a.y, dz = b.z - a.z;
                if (PER) {
                    double Sx, Sy, Sz;
                    int ky;
                    image_shift(G, dx, dy, dz, Sx, Sy, Sz, ky);
                    dx = dx + Sx;
                    dy = dy + Sy;
                    dz = dz + Sz;
                }
                if (touching(dx, dy, dz, ri + (double)meta_r(b.w))) {
                    const uint32_t pj = meta_pid(b.w);
                    int k = (int)cnt;
                    while (k > 0 && pid_at(k - 1) > pj) {
                        pid_at(k) = pid_at(k - 1);
                        s_j[k * DTILE + t] = s_j[(k - 1) * DTILE + t];
                        --k;
                    }
                    pid_at(k) = pj;
                    s_j[k * DTILE + t] = jj[m];
                    ++cnt;
                }
            }
        }
    }
    // box faces last, in face order (their ids sort after every particle)
    if (G.walls && cnt <= KMAX) {
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            if (!(G.walls & (1u << f))) continue;
            const int ax = f >> 1;
            const double pc = ax == 0 ? a.x : (ax == 1 ? a.y : a.z);
            const double dist = (f & 1) ? G.hi[ax] - pc : pc - G.lo[ax];
            if (dist < ri) {
                if (cnt < KMAX) {
                    pid_at((int)cnt) = FACE + (uint32_t)f;
                    s_j[cnt * DTILE + t] = FACE + (uint32_t)f;
                }
                ++cnt;
            }
        }
    }
    // then the extra walls, in order
    for (uint32_t k = 0; k < nxw && cnt <= KMAX; ++k) {
        if (wall_touch(xw[k], a.x, a.y, a.z, ri)) {
            if (cnt < KMAX) {
                pid_at((int)cnt) = FACE + 6u + k;
                s_j[cnt * DTILE + t] = FACE + 6u + k;
            }
            ++cnt;
        }
    }
    if (cnt > KMAX) {
        atomicOr(&P.st->err, ERR_ROW);
        cnt = 0;
    }
    return cnt;
}

// Row lengths of the workgroup's lanes into one contiguous region of the
// contact list (the tile's own region: no device-wide counter), partner
// positions from the lanes' columns of s_j.  Called by every lane.
template <int KMAX>
__device__ __forceinline__ void write_rows(const PoolView& P, uint32_t tile, int t, uint32_t i,
                                           bool act, uint32_t cnt, const uint32_t* s_j,
                                           uint32_t* s_excl, uint32_t* s_w, uint32_t* s_base,
                                           uint2* __restrict__ rows,
                                           uint32_t* __restrict__ col_j, uint32_t slots) {
    uint32_t total;
    const uint32_t excl = block_excl_scan<DTILE / 64>(cnt, s_w, total);
    s_excl[t] = excl;
    if (t == 0) {
        // the workgroup's own region of the contact list: no device-wide counter
        s_excl[DTILE] = total;
        uint32_t base = tile * (uint32_t)DTILE * slots;
        if (total > (uint32_t)DTILE * slots) {
            atomicOr(&P.st->err, ERR_CAPACITY);
            atomicMax(&P.st->need, total);
            base = 0xFFFFFFFFu;
        } else {
            P.ts[tile].m_step = total;
        }
        *s_base = base;
    }
    __syncthreads();
    const uint32_t base = *s_base;
    if (base == 0xFFFFFFFFu) return;
    if (act) rows[i] = make_uint2(base + excl, cnt);
    for (uint32_t q = t; q < total; q += DTILE) {
        const int o = owner_of<DTILE>(s_excl, q);
        col_j[base + q] = s_j[(q - s_excl[o]) * DTILE + o];
    }
}

// One lane per particle, DTILE consecutive particles (cell order) per
// workgroup; the lane walks the candidate ranges of its particle.
//
// Candidates are read as one 16-byte FP32 record each (position relative to
// the box corner, radius) and pre-filtered with a margin that covers the
// float rounding, so the pre-filter never rejects a pair that touches in FP64.
// The survivors (the contacts plus rare near misses) are kept in LDS and then
// take the exact FP64 test on the original positions, four loads in flight,
// which keeps the contact set exactly the FP64 one.  Hits go into the lane's
// LDS row in partner-id order; box faces come last; the workgroup compacts its
// rows into its own region of the contact list.
template <int KMAX, bool PER>
__global__ __launch_bounds__(DTILE) void k_detect(PoolView P, const Job* __restrict__ jobs,
                                                  SortedPos xr,
                                                  const float4* __restrict__ xf,
                                                  const uint2* __restrict__ cells,
                                                  uint2* __restrict__ rows,
                                                  uint32_t* __restrict__ col_j, uint32_t slots) {
    constexpr int NW = DTILE / 64;
    // survivors, then contacts, of each lane; slot KMAX takes the writes of
    // a lane whose row is already full
    __shared__ uint32_t s_j[(KMAX + 1) * DTILE];
    // this lane's non-empty candidate ranges (9 rows, plus the wrapped x
    // neighbour of each row with periodic boxes, plus a sentinel) during the
    // candidate walk; afterwards the same 8-byte slots (same lane, same
    // stride, so no lane ever touches another lane's slots) hold the partner
    // ids of the lane's contacts
    constexpr int NWIN = PER ? 18 : 9;
    constexpr int NSLOT = (NWIN + 1) > KMAX ? (NWIN + 1) : KMAX;
    __shared__ uint2 s_winpid[NSLOT * DTILE];
    uint2* const s_win = s_winpid;
    __shared__ uint32_t s_excl[DTILE + 1];
    __shared__ uint32_t s_w[NW];
    __shared__ uint32_t s_base, s_flag;
    Status* st = P.st;
    if (skip_if_error(st, &s_flag)) return;

    const int t = threadIdx.x;
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
    uint32_t jb;
    const Job* Jp = tile_job(jobs, P, tile, jb);
    if (!Jp) return;
    const Job& J = *Jp;
    const Geo& G = J.g;
    const float margin = J.margin;
    cells += J.cell_base;
    const uint32_t i = tile * DTILE + t;
    const bool act = i < J.p0 + J.n;

    uint32_t cnt = 0;
    uint32_t nw = 0;
    if (act) {
        const double4 a = xr[i];
        const double ri = (double)meta_r(a.w);
        nw = candidate_ranges<PER>(G, a, ri, cells, s_win + t, DTILE);

        // FP32 pre-filter: never rejects a pair that touches in FP64 (NaN
        // records of particles far from the box always pass)
        const PreFilter<PER> pre(G, a, margin);
        // pass 1: one flat loop over all candidates of all ranges with the
        // records of the next candidates already in flight; survivors go
        // unsorted into the row buffer.  The walk over the ranges is
        // branch-free: the range after the current one is always read ahead
        // from LDS, and a sentinel range ends the walk.  A finished lane keeps
        // loading its own record (always in bounds) and ignores it.
        constexpr uint32_t NONE = 0xFFFFFFFFu;
        uint32_t sc = 0;
        if (nw > 0) {
            s_win[nw * DTILE + t] = make_uint2(NONE, NONE);
            uint32_t w = 0;
            uint2 rg = s_win[t];
            uint2 rn = s_win[DTILE + t];
            uint32_t j = rg.x;  // next candidate to fetch
            auto next = [&]() -> uint32_t {
                const uint32_t c = j;
                const bool live = c != NONE;
                const bool sw = live && c + 1 == rg.y;
                j = !live ? NONE : (sw ? rn.x : c + 1);
                rg.y = sw ? rn.y : rg.y;
                w += sw ? 1u : 0u;
                rn = s_win[min(w + 1, nw) * DTILE + t];
                return c;
            };
            // four slots in rotation: a slot's record is tested, then the slot
            // is refilled with the candidate four places ahead, so three loads
            // stay in flight while a record is tested
            uint32_t j0 = next(), j1 = next(), j2 = next(), j3 = next();
            // every load index is checked against the position capacity
            // (NONE is above it): an index that is not a position is never read
            const uint32_t nsz = P.ns;
            float4 q0 = xf[j0 < nsz ? j0 : i], q1 = xf[j1 < nsz ? j1 : i];
            float4 q2 = xf[j2 < nsz ? j2 : i], q3 = xf[j3 < nsz ? j3 : i];
#define DEM_PRE_STEP(Q, JQ)                                        \
    {                                                              \
        if (JQ == NONE) break;                                     \
        const bool hit = (JQ != i) & pre(Q);                       \
        s_j[min(sc, (uint32_t)KMAX) * DTILE + t] = JQ;             \
        sc += hit ? 1u : 0u;                                       \
        JQ = next();                                               \
        Q = xf[JQ < nsz ? JQ : i];                                 \
    }
            for (;;) {
                DEM_PRE_STEP(q0, j0)
                DEM_PRE_STEP(q1, j1)
                DEM_PRE_STEP(q2, j2)
                DEM_PRE_STEP(q3, j3)
            }
#undef DEM_PRE_STEP
        }
        cnt = detect_row<KMAX, PER>(P, G, a, ri, i, t, sc, nw,
                                    [&](uint32_t w2) { return s_win[w2 * DTILE + t]; }, xr, s_j,
                                    s_winpid + t, DTILE, J.xw, J.nxw);
    }
    write_rows<KMAX>(P, tile, t, i, act, cnt, s_j, s_excl, s_w, &s_base, rows, col_j, slots);
}

// ------------------------------------------------------------ half detect
// Wide scan of one large particle ("big": radius above the job's cut) by the
// whole wavefront (two-level contact search).  The one-cell stencil of the
// half search only holds partners of particles no larger than the cut; a big
// particle instead scans every cell within two cells of its own (cells are
// at least as wide as its largest contact distance halved) and enters each
// contact it finds in both lists.  A pair of two big particles is entered by
// the one at the lower position.  Lane l < 25 forms row l of the 5 x 5 rows
// of the stencil (its cells within reach, at most two contiguous ranges when
// the row wraps around a periodic x axis); the wavefront then tests the
// concatenated ranges 64 candidates at a time with the exact FP64 predicate.
// s_w: this wavefront's 64 words x 4 of scratch in LDS (column lane,
// stride DTILE).
template <bool PER, typename Append>
__device__ __forceinline__ void wide_scan(const Geo& G, const uint2* __restrict__ cells,
                                          SortedPos xr, uint32_t nsz,
                                          const double4& b, uint32_t bi, int lane,
                                          uint32_t* s_w, Append append) {
    const int nx = G.nc[0], ny = G.nc[1], nz = G.nc[2];
    const bool px = PER && (G.periodic & 1u), py = PER && (G.periodic & 2u),
               pz = PER && (G.periodic & 4u), le = PER && G.le;
    const double rb = (double)meta_r(b.w);
    const uint32_t bpid = meta_pid(b.w);
    const double reach = rb + G.reach_big;
    const int cy = cell_coord(G, b.y, 1), cz = cell_coord(G, b.z, 2);
    uint32_t lo1 = 0, n1 = 0, lo2 = 0, n2 = 0;
    if (lane < 25) {
        const int oy = lane % 5 - 2, oz = lane / 5 - 2;
        int y = cy + oy, z = cz + oz, ky = 0;
        bool ok = true;
        if (y < 0 || y >= ny) {
            if (!py) ok = false;
            ky = y < 0 ? -1 : 1;
            y -= ky * ny;
        }
        if (z < 0 || z >= nz) {
            if (!pz) ok = false;
            z = z < 0 ? z + nz : z - nz;
        }
        // squared gaps to the row's (y, z) slab, in the unwrapped frame
        double gy = 0.0, gz = 0.0;
        if (oy > 0) gy = G.lo[1] + (double)(cy + oy) * G.cw[1] - b.y;
        if (oy < 0) gy = b.y - (G.lo[1] + (double)(cy + oy + 1) * G.cw[1]);
        if (oz > 0) gz = G.lo[2] + (double)(cz + oz) * G.cw[2] - b.z;
        if (oz < 0) gz = b.z - (G.lo[2] + (double)(cz + oz + 1) * G.cw[2]);
        gy = fmax(gy, 0.0);
        gz = fmax(gz, 0.0);
        const double rx2 = reach * reach - gy * gy - gz * gz;
        if (ok && rx2 > 0.0) {
            const double rx = sqrt(rx2);
            // across a sheared y boundary the partner row is offset along x
            const double bx = le && ky != 0 ? b.x - (double)ky * G.le_shift : b.x;
            const double lim = 4.0 * (double)nx;
            double fl = floor((bx - rx - G.lo[0]) * G.inv_cell[0]);
            double fh = floor((bx + rx - G.lo[0]) * G.inv_cell[0]);
            double fc = floor((bx - G.lo[0]) * G.inv_cell[0]);
            fl = fmin(fmax(fl, -lim), lim);  // also NaN -> -lim
            fh = fmin(fmax(fh, -lim), lim);
            fc = fmin(fmax(fc, -lim), lim);
            int xl = (int)fl, xh = (int)fh;
            int xc = (int)fc;
            if (px) {
                // the window relative to the cell of the x-aligned image in [0, nx)
                int m = xc % nx;
                m = m < 0 ? m + nx : m;
                xl -= xc - m;
                xh -= xc - m;
                xc = m;
            }
            if (!px) {
                // cells clamp coordinates outside the box into the border cells
                xc = cell_coord(G, b.x, 0);
                xl = xl < 0 ? 0 : (xl > nx - 1 ? nx - 1 : xl);
                xh = xh < 0 ? 0 : (xh > nx - 1 ? nx - 1 : xh);
            }
            xl = xl < xc - 2 ? xc - 2 : xl;
            xh = xh > xc + 2 ? xc + 2 : xh;
            const uint32_t row = ((uint32_t)z * (uint32_t)ny + (uint32_t)y) * (uint32_t)nx;
            uint32_t a1 = 0xFFFFFFFFu, e1 = 0u, a2 = 0xFFFFFFFFu, e2 = 0u;
            // the window's (at most 5) cell bounds are all loaded before any
            // is merged; a window of at most 5 cells on a periodic axis of at
            // least 5 wraps at most once, and its wrapped cells form the
            // second range
            uint2 cb[5];
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                const int x = xc - 2 + k;
                const int xw = x < 0 ? x + nx : (x >= nx ? x - nx : x);
                const bool in = x >= xl && x <= xh && xw >= 0 && xw < nx;
                cb[k] = in ? cells[row + (uint32_t)xw] : make_uint2(0u, 0u);
            }
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                const int x = xc - 2 + k;
                if (x < 0 || x >= nx) merge_range(cb[k], a2, e2); else merge_range(cb[k], a1, e1);
            }
            if (e1 > a1) { lo1 = a1; n1 = e1 - a1; }
            if (e2 > a2) { lo2 = a2; n2 = e2 - a2; }
        }
    }
    // exclusive prefix of the rows' candidate counts over the wavefront
    const uint32_t cnt = n1 + n2;
    uint32_t inc = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_up(inc, o, 64);
        if (lane >= o) inc += u;
    }
    const uint32_t total = __shfl(inc, 63, 64);
    s_w[0] = inc - cnt;
    s_w[DTILE] = lo1;
    s_w[2 * DTILE] = n1;
    s_w[3 * DTILE] = lo2;
    __builtin_amdgcn_wave_barrier();
    uint32_t* const s0 = s_w - lane;  // lane 0's column of this wavefront
    for (uint32_t k0 = 0; k0 < total; k0 += 64) {
        const uint32_t q = k0 + (uint32_t)lane;
        if (q < total) {
            // the row whose candidates hold q: the last of rows 0..24 with
            // exclusive prefix <= q
            int lo = 0, hi = 24;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s0[mid] <= q) lo = mid; else hi = mid - 1;
            }
            const uint32_t off = q - s0[lo];
            const uint32_t m1 = s0[2 * DTILE + lo];
            const uint32_t j = off < m1 ? s0[DTILE + lo] + off : s0[3 * DTILE + lo] + (off - m1);
            if (j != bi && j < nsz) {
                const double4 c = xr[j];
                const float rj = meta_r(c.w);
                // a pair of two big particles: entered from the lower position
                if (!(rj > G.rcut && j < bi)) {
                    double dx = c.x - b.x, dy = c.y - b.y, dz = c.z - b.z;
                    if (PER) {
                        double Sx, Sy, Sz;
                        int ky;
                        image_shift(G, dx, dy, dz, Sx, Sy, Sz, ky);
                        dx = dx + Sx;
                        dy = dy + Sy;
                        dz = dz + Sz;
                    }
                    if (touching(dx, dy, dz, rb + (double)rj)) {
                        append(bi, j, meta_pid(c.w));
                        append(j, bi, bpid);
                    }
                }
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
}

// Contact search that tests each pair once: the lane of a particle walks the
// upper half of its cell stencil (the half-shell of candidate_ranges, about
// 13.5 of the 27 cells for every particle alike, so the lanes of a wave stay
// balanced).  The contact test is symmetric in the two particles (the image
// shift is odd in the separation, the distance test even), so every touching
// pair is found exactly once, from one of its two particles.  Each contact goes into
// both particles' adjacency lists as (position, partner id) with an atomic
// slot counter per particle; slot k of every particle's list is one array
// (adj[k * ns + p], KMAX slots), so the lists of neighbouring particles share
// cache lines and are read coalesced.  Box faces and extra walls go into the
// particle's own list.  The force kernel (k_force with HK) turns the lists
// into rows ordered by partner id: the rows of the full search.
//
// Two-level search: when a job has particles larger than its radius cut
// G.rcut (a few per cent of a polydisperse job), its cells are sized for the
// cut instead of the largest radius, which shrinks every particle's stencil;
// the lanes skip those "big" particles (as partners and as walkers), and each
// wavefront then runs the wide scan of its own big particles.
template <int KMAX, bool PER>
__global__ __launch_bounds__(DTILE) void k_detect_half(PoolView P, const Job* __restrict__ jobs,
                                                       SortedPos xr,
                                                       const float4* __restrict__ xf,
                                                       const uint2* __restrict__ cells,
                                                       uint32_t* __restrict__ deg,
                                                       uint2* __restrict__ adj) {
    // survivors of the FP32 pre-filter, SB per lane (slot SB takes the
    // writes of a lane whose buffer is full; such a lane re-walks with the
    // exact test and enters its contacts directly, so the buffer need not
    // hold a whole row); afterwards the wide scans' row table
    constexpr int SB = 8;
    __shared__ uint32_t s_j[(SB + 1) * DTILE];
    // the half stencil has 5 rows: at most 5 ranges (10 with the wrapped x
    // neighbours of a periodic box), plus the sentinel
    constexpr int NWIN = PER ? 10 : 5;
    __shared__ uint2 s_win[(NWIN + 1) * DTILE];
    __shared__ uint32_t s_flag;
    Status* st = P.st;
    const int t = threadIdx.x;
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t i = tile * DTILE + t;
    // the own record is read before the error check and the job lookup (it
    // is a position whatever the tile holds)
    const double4 a = xr[i];
    if (skip_if_error(st, &s_flag)) return;
    uint32_t jb;
    const Job* Jp = tile_job(jobs, P, tile, jb);
    if (!Jp) return;
    const Job& J = *Jp;
    const Geo& G = J.g;
    cells += J.cell_base;
    // lanes past the job's last particle stay (the wide scan needs every
    // lane of the wavefront) but search nothing
    const bool valid = i < J.p0 + J.n;
    const uint32_t nsz = P.ns;
    auto append = [&](uint32_t p, uint32_t q, uint32_t pid) {
        const uint32_t k = atomicAdd(&deg[p], 1u);
        if (k < (uint32_t)KMAX) adj[(size_t)k * nsz + p] = make_uint2(q, pid);
    };
    const double ri = (double)meta_r(a.w);
    const uint32_t pi = meta_pid(a.w);
    const bool big = valid && meta_r(a.w) > G.rcut;
    const uint32_t nw = (valid && !big) ?
        candidate_ranges<PER, true>(G, a, ri, cells, s_win + t, DTILE, nullptr, i) : 0u;
    // In a periodic box a particle whose cell is at least one cell away from
    // every periodic boundary (on axes of 5 cells or more) has all its
    // candidates within 2 cells, less than 0.4 box lengths: the image shift
    // is zero for all of them.  A wave whose particles are all such takes
    // the plain filter and the plain exact test, with the same results.
    bool plain = true;
    if (PER) {
        const int c[3] = {cell_coord(G, a.x, 0), cell_coord(G, a.y, 1), cell_coord(G, a.z, 2)};
#pragma unroll
        for (int ax = 0; ax < 3; ++ax)
            if (G.periodic & (1u << ax))
                plain = plain && G.nc[ax] >= 5 && c[ax] >= 1 && c[ax] <= G.nc[ax] - 2;
        plain = __all(plain) != 0;
    }
    const PreFilter<PER> pre(G, a, J.margin);
    const PreFilter<false> pre0(G, a, J.margin);
    const PreFilter<false, false> pre1(G, a, J.margin);
    constexpr uint32_t NONE = 0xFFFFFFFFu;
    uint32_t sc = 0;
    auto walk = [&](const auto& filt) {
        // the plain kernel's walk: branch-free over the ranges, four records
        // in flight.  After the last range the walk stays on the particle's
        // own position (a range of one entry behind the last), so every
        // index it loads is a position; a count of the candidates left
        // masks the slots past the end.
        if (nw == 0) return;
        uint32_t left = 0;
        for (uint32_t w2 = 0; w2 < nw; ++w2) {
            const uint2 r2 = s_win[w2 * DTILE + t];
            left += r2.y - r2.x;
        }
        s_win[nw * DTILE + t] = make_uint2(i, i + 1);
        uint32_t w = 0;
        uint2 rg = s_win[t];
        uint2 rn = s_win[DTILE + t];
        uint32_t j = rg.x;
        auto next = [&]() -> uint32_t {
            const uint32_t c = j;
            const bool sw = c + 1 == rg.y;
            j = sw ? rn.x : c + 1;
            rg.y = sw ? rn.y : rg.y;
            w += sw ? 1u : 0u;
            rn = s_win[min(w + 1, nw) * DTILE + t];
            return c;
        };
        uint32_t j0 = next(), j1 = next(), j2 = next(), j3 = next();
        float4 q0 = xf[j0], q1 = xf[j1], q2 = xf[j2], q3 = xf[j3];
        // the four slots hold consecutive candidates, the oldest in slot 0
#define DEM_HALF_STEP(Q, JQ, S)                                    \
    {                                                              \
        const bool hit = (left > S) & filt(Q);                     \
        s_j[min(sc, (uint32_t)SB) * DTILE + t] = JQ;               \
        sc += hit ? 1u : 0u;                                       \
        JQ = next();                                               \
        Q = xf[JQ];                                                \
    }
        while (left > 0) {
            DEM_HALF_STEP(q0, j0, 0u)
            DEM_HALF_STEP(q1, j1, 1u)
            DEM_HALF_STEP(q2, j2, 2u)
            DEM_HALF_STEP(q3, j3, 3u)
            left = left > 4u ? left - 4u : 0u;
        }
#undef DEM_HALF_STEP
    };
    // a one-level job (no particle above the cut) skips the radius test
    if ((!PER || plain) && G.nbig == 0)
        walk(pre1);
    else if (!PER || plain)
        walk(pre0);
    else
        walk(pre);
    if (sc > SB) {
        // more survivors than the buffer holds: walk the candidates again
        // with the exact FP64 test and enter each contact at once (a list
        // that outgrows its slots is reported by the force kernel)
        for (uint32_t w2 = 0; w2 < nw; ++w2) {
            const uint2 rg2 = s_win[w2 * DTILE + t];
            for (uint32_t jx = rg2.x; jx < rg2.y; ++jx) {
                if (jx >= nsz) continue;
                const double4 b = xr[jx];
                if (meta_r(b.w) > G.rcut) continue;  // the wide scan's pair
                double dx = b.x - a.x, dy = b.y - a.y, dz = b.z - a.z;
                if (PER && !plain) {
                    double Sx, Sy, Sz;
                    int ky;
                    image_shift(G, dx, dy, dz, Sx, Sy, Sz, ky);
                    dx = dx + Sx;
                    dy = dy + Sy;
                    dz = dz + Sz;
                }
                if (touching(dx, dy, dz, ri + (double)meta_r(b.w))) {
                    append(i, jx, meta_pid(b.w));
                    append(jx, i, pi);
                }
            }
        }
    } else {
        // exact FP64 test of the survivors, four loads in flight
        for (uint32_t k0 = 0; k0 < sc; k0 += 4) {
            uint32_t jj[4];
            double4 bb[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) jj[m] = k0 + m < sc ? s_j[(k0 + m) * DTILE + t] : NONE;
#pragma unroll
            for (int m = 0; m < 4; ++m) bb[m] = xr[jj[m] < nsz ? jj[m] : i];
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                if (jj[m] >= nsz) continue;
                const double4 b = bb[m];
                double dx = b.x - a.x, dy = b.y - a.y, dz = b.z - a.z;
                if (PER && !plain) {
                    double Sx, Sy, Sz;
                    int ky;
                    image_shift(G, dx, dy, dz, Sx, Sy, Sz, ky);
                    dx = dx + Sx;
                    dy = dy + Sy;
                    dz = dz + Sz;
                }
                if (touching(dx, dy, dz, ri + (double)meta_r(b.w))) {
                    append(i, jj[m], meta_pid(b.w));
                    append(jj[m], i, pi);
                }
            }
        }
    }
    if (valid) {
        // box faces, then extra walls: the particle's own list
        if (G.walls) {
            for (int f = 0; f < 6; ++f) {
                if (!(G.walls & (1u << f))) continue;
                const int ax = f >> 1;
                const double pc = ax == 0 ? a.x : (ax == 1 ? a.y : a.z);
                const double dist = (f & 1) ? G.hi[ax] - pc : pc - G.lo[ax];
                if (dist < ri) append(i, FACE + (uint32_t)f, FACE + (uint32_t)f);
            }
        }
        for (uint32_t k = 0; k < J.nxw; ++k)
            if (wall_touch(J.xw[k], a.x, a.y, a.z, ri)) append(i, FACE + 6u + k, FACE + 6u + k);
    }
    if (G.nbig) {
        // the wavefront's big particles, one at a time, by all its lanes
        const int lane = t & 63;
        unsigned long long bal = __ballot(big);
        while (bal) {
            const int src = __ffsll((long long)bal) - 1;
            bal &= bal - 1ull;
            double4 b;
            b.x = __shfl(a.x, src, 64);
            b.y = __shfl(a.y, src, 64);
            b.z = __shfl(a.z, src, 64);
            b.w = __shfl(a.w, src, 64);
            const uint32_t bi = tile * DTILE + (uint32_t)(t - lane) + (uint32_t)src;
            wide_scan<PER>(G, cells, xr, nsz, b, bi, lane, s_j + t, append);
        }
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
// Terms of one contact of the particle at a (state a0, a1, a2 = v_x v_y,
// v_z w_x, w_y w_z; material mi) with `code`, a partner's sorted position or
// a box face: unit normal towards the partner, overlap, relative velocity of
// the centres, the radius-weighted sum of angular velocities, reduced radius
// and mass, the partner's material and id.  A face has infinite radius and
// mass and the particle's own material.
template <typename R>
struct PairTerms {
    R nx, ny, nz, dn, vx, vy, vz, rwx, rwy, rwz, rs, ms;
    int mj;
    uint32_t pid;
};

template <typename R>
__device__ __forceinline__ PairTerms<R> pair_terms(
    const Geo& G, const MatTable* __restrict__ mt, uint32_t code, const double4& a,
    const double2& a0, const double2& a1, const double2& a2, int mi,
    const double4* __restrict__ xr_x, const double2* __restrict__ vw,
    const uint8_t* __restrict__ mat, const uint32_t* __restrict__ perm, uint32_t ns,
    const dem_wall* __restrict__ xw) {
    PairTerms<R> p;
    const R ri = (R)meta_r(a.w);
    const double rid = (double)meta_r(a.w);
    const R mass_i = (R)(mt->mass_pref[mi] * rid * rid * rid);
    if (code < FACE) {
        // the partner's records, all in the state buffer read, through the
        // permutation
        const uint32_t j = code;
        const uint32_t qj = perm[j];
        const double4 b = xr_x[qj];
        const double2 b0 = vw[qj], b1 = vw[ns + qj], b2 = vw[2 * (size_t)ns + qj];
        p.mj = mat ? mat[qj] : 0;
        p.pid = meta_pid(b.w);
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
        // the predicate's own d2 (same operations, no fused multiply-add):
        // d2 < s^2 holds here exactly as it did in the contact search, so
        // with a correctly rounded square root d <= s and the overlap is
        // never negative; the clamp keeps sqrt(dn) finite even so.  The
        // overlap is taken in FP64 in both precisions (s - d cancels), the
        // normal in the force precision.
        const double d2 = dist2(dx, dy, dz);
        const double s = rid + rjd;
        const double d = sqrt(d2);
        p.dn = (R)fmax(s - d, 0.0);
        if (sizeof(R) == 8) {
            p.nx = (R)(dx / d);
            p.ny = (R)(dy / d);
            p.nz = (R)(dz / d);
        } else {
            const float inv = 1.0f / (float)d;
            p.nx = (R)((float)dx * inv);
            p.ny = (R)((float)dy * inv);
            p.nz = (R)((float)dz * inv);
        }
        p.vx = (R)((a0.x - b0.x) - (double)ky * G.le_dv);
        p.vy = (R)(a0.y - b0.y);
        p.vz = (R)(a1.x - b1.x);
        p.rwx = ri * (R)a1.y + rj * (R)b1.y;
        p.rwy = ri * (R)a2.x + rj * (R)b2.x;
        p.rwz = ri * (R)a2.y + rj * (R)b2.y;
        p.rs = ri * rj / (ri + rj);
        const R mass_j = (R)(mt->mass_pref[p.mj] * rjd * rjd * rjd);
        p.ms = mass_i * mass_j / (mass_i + mass_j);
    } else {
        const int f = (int)(code - FACE), ax = f >> 1;
        p.pid = code;
        p.mj = mi;
        if (f < 6) {
            const double q = ax == 0 ? a.x : (ax == 1 ? a.y : a.z);
            const double dist = (f & 1) ? G.hi[ax] - q : q - G.lo[ax];
            const R sg = (f & 1) ? (R)1 : (R)-1;
            p.nx = ax == 0 ? sg : (R)0;
            p.ny = ax == 1 ? sg : (R)0;
            p.nz = ax == 2 ? sg : (R)0;
            p.dn = (R)(rid - dist);
        } else {
            // extra wall: normal from the centre to the wall's closest point
            const dem_wall& W = xw[f - 6];
            double wx, wy, wz;
            const double d = sqrt(wall_gap(W, a.x, a.y, a.z, wx, wy, wz));
            if (!(d > 0.0)) {
                // centre on the rectangle: its normal u x v
                wx = W.u[1] * W.v[2] - W.u[2] * W.v[1];
                wy = W.u[2] * W.v[0] - W.u[0] * W.v[2];
                wz = W.u[0] * W.v[1] - W.u[1] * W.v[0];
                const double l = sqrt(wx * wx + wy * wy + wz * wz);
                p.nx = (R)(wx / l);
                p.ny = (R)(wy / l);
                p.nz = (R)(wz / l);
            } else {
                p.nx = (R)(wx / d);
                p.ny = (R)(wy / d);
                p.nz = (R)(wz / d);
            }
            p.dn = (R)fmax(rid - d, 0.0);
        }
        p.vx = (R)a0.x;
        p.vy = (R)a0.y;
        p.vz = (R)a1.x;
        p.rwx = ri * (R)a1.y;
        p.rwy = ri * (R)a2.x;
        p.rwz = ri * (R)a2.y;
        p.rs = ri;
        p.ms = mass_i;
    }
    return p;
}

// Tangential displacement carried by the pair with partner id `pid` in the
// previous step's row `orw` of the particle; zero for a new contact.  Returns
// whether the pair was found.  Rows of the split path are sorted by partner
// id, which ends the search early; rows of the fused path are in the order
// the candidates were visited.
template <bool SORTED>
__device__ __forceinline__ bool history_of(uint2 orw, uint32_t pid,
                                           const uint32_t* __restrict__ tab_pid_old,
                                           const double* __restrict__ tab_dt_old, uint64_t cap,
                                           double& dtx, double& dty, double& dtz) {
    dtx = dty = dtz = 0.0;
    // partner ids read four at a time, so that a row's search takes one
    // memory round trip rather than one per entry
    const uint32_t end = orw.x + orw.y;
    for (uint32_t k0 = orw.x; k0 < end; k0 += 4) {
        uint32_t pk[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) pk[m] = k0 + m < end ? tab_pid_old[k0 + m] : 0u;
        int hit = -1;
        bool past = false;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const bool in = k0 + m < end;
            if (hit < 0 && !past && in && pk[m] == pid) hit = m;
            if (SORTED && in && pk[m] > pid) past = true;
        }
        if (hit >= 0) {
            const uint32_t k = k0 + (uint32_t)hit;
            dtx = tab_dt_old[k];
            dty = tab_dt_old[(size_t)cap + k];
            dtz = tab_dt_old[2 * (size_t)cap + k];
            return true;
        }
        if (past) break;
    }
    return false;
}

// Sort input of a position that keeps its place (ghost slot, idle tile):
// with the merge sort (movers given) only its key before the step, which is
// also its key after; with the radix sort its key and index.
__device__ __forceinline__ void fixed_sort_input(uint32_t* __restrict__ keys,
                                                 uint32_t* __restrict__ vals,
                                                 uint32_t* __restrict__ oldkeys, bool merge,
                                                 uint32_t i, uint32_t key) {
    if (merge) {
        oldkeys[i] = key;
    } else {
        keys[i] = key;
        vals[i] = i;
    }
}

// A tile whose job is not running: keys that keep every position of the
// tile in place; a finished job's state is carried over into the buffer
// written.
__device__ __forceinline__ void idle_tile(const PoolView& P, const Job* __restrict__ jobs,
                                          uint32_t tile, uint32_t jb, int t,
                                          const double4* __restrict__ xr_x,
                                          const double2* __restrict__ vw,
                                          const uint8_t* __restrict__ mat,
                                          double4* __restrict__ xr_b, double2* __restrict__ vw_b,
                                          uint8_t* __restrict__ mat_b,
                                          const uint32_t* __restrict__ perm,
                                          uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
                                          uint32_t* __restrict__ oldkeys, bool movers) {
    const uint32_t p0 = tile * TILE, ns = P.ns;
    fixed_sort_input(keys, vals, oldkeys, movers, p0 + t, tile_key_of(P, tile) | P.lmask);
    if (jb != NO_JOB) {
        const uint32_t i = p0 + t;
        if (i < jobs[jb].p0 + jobs[jb].n) {
            const uint32_t q = perm[i];
            xr_b[i] = xr_x[q];
            vw_b[i] = vw[q];
            vw_b[ns + i] = vw[ns + q];
            vw_b[2 * (size_t)ns + i] = vw[2 * (size_t)ns + q];
            if (mat_b) mat_b[i] = mat[q];
        }
    }
}

// The end of a step for the TILE particles of a running tile, called by every
// lane of the workgroup: with `churn`, the churn counters (and, when `m` is
// given, the contact count) into the tile's own slot; per-particle totals, gravity and the
// semi-implicit Euler update in FP64 (section 3.4, "ForceGravity" and
// "Integrate") into the buffer written; the new cell key ("CalcHash") and the
// sort's input: with the merge sort (movers given) the key before the step
// and the cell-change list, with the radix sort the key and index.  With
// clear_cells and the radix sort, the first particle of each old cell also
// empties that cell's bounds (the reorder writes those of the new order); the
// merge sort empties the old cells of the particles that changed cell, the
// only cells that can be left empty.
template <typename R>
__device__ __forceinline__ void finish_tile(
    const PoolView& P, const Geo& G, const MatTable* __restrict__ mt, uint32_t tile, uint32_t jb,
    int t, uint32_t i, uint32_t n, const double4& a, const double2& a0, const double2& a1,
    const double2& a2, int mi, const R* acc, bool churn, uint32_t matched, uint32_t old,
    const uint32_t* m, double4* __restrict__ xr_b, double2* __restrict__ vw_b, uint8_t* __restrict__ mat_b,
    uint2* __restrict__ cells, bool clear_cells, uint32_t* __restrict__ keys,
    uint32_t* __restrict__ vals, R* __restrict__ fo, uint32_t* __restrict__ oldkeys,
    uint2* __restrict__ movers) {
    __shared__ uint32_t s_red[6];
    const uint32_t ns = P.ns;
    Status* st = P.st;
    if (churn) {
        uint32_t mv = matched, ov = old, cv = m ? *m : 0u;
        for (int o = 32; o > 0; o >>= 1) {
            mv += __shfl_down(mv, o, 64);
            ov += __shfl_down(ov, o, 64);
            if (m) cv += __shfl_down(cv, o, 64);
        }
        if ((t & 63) == 0) {
            s_red[3 * (t >> 6)] = mv;
            s_red[3 * (t >> 6) + 1] = ov;
            s_red[3 * (t >> 6) + 2] = cv;
        }
        __syncthreads();
        if (t == 0) {
            P.ts[tile].matched_step = s_red[0] + s_red[3];
            P.ts[tile].old_step = s_red[1] + s_red[4];
            if (m) P.ts[tile].m_step = s_red[2] + s_red[5];
        }
    }
    bool moved = false;
    uint32_t newkey = 0;
    if (i < n) {
        const double r = (double)meta_r(a.w);
        const double mass = mt->mass_pref[mi] * r * r * r;
        const double I = 0.4 * mass * r * r;
        const double Fx = (double)acc[0] + mass * G.g[0];
        const double Fy = (double)acc[1] + mass * G.g[1];
        const double Fz = (double)acc[2] + mass * G.g[2];
        double vx = a0.x + G.dt * Fx / mass;
        double vy = a0.y + G.dt * Fy / mass;
        double vz = a1.x + G.dt * Fz / mass;
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
        if (!finite) atomicOr(&P.job_fail[jb], 1u);
        xr_b[i] = make_double4(x, y, z, a.w);
        vw_b[i] = make_double2(vx, vy);
        vw_b[ns + i] = make_double2(vz, wx);
        vw_b[2 * (size_t)ns + i] = make_double2(wy, wz);
        if (mat_b) mat_b[i] = (uint8_t)mi;
        newkey = tile_key_of(P, tile) | cell_key(G, x, y, z);
        if (!movers) {
            keys[i] = newkey;
            vals[i] = i;
        }
        if (fo) {
            fo[i] = (R)Fx;
            fo[ns + i] = (R)Fy;
            fo[2 * (size_t)ns + i] = (R)Fz;
            fo[3 * (size_t)ns + i] = acc[3];
            fo[4 * (size_t)ns + i] = acc[4];
            fo[5 * (size_t)ns + i] = acc[5];
        }
        const uint32_t okey = cell_key(G, a.x, a.y, a.z);
        if (clear_cells && !movers) {
            const uint32_t lin = key_lin(G, okey);
            if (cells[lin].x == i) cells[lin] = make_uint2(0, 0);
        }
        if (movers) {
            const uint32_t oldkey = tile_key_of(P, tile) | okey;
            oldkeys[i] = oldkey;
            moved = newkey != oldkey;
        }
    }
    if (movers) {
        // the particles that changed cell join the step's mover list: one
        // reservation per workgroup that has any
        __shared__ uint32_t s_mv[2], s_mvbase;
        const int lane = t & 63, w = t >> 6;
        const unsigned long long bal = __ballot(moved);
        if (lane == 0) s_mv[w] = (uint32_t)__popcll(bal);
        __syncthreads();
        if (t == 0) {
            const uint32_t tot = s_mv[0] + s_mv[1];
            uint32_t b = 0;
            if (tot) {
                b = atomicAdd(&st->movers, tot);
                if (b + tot > MAX_MOVERS) {
                    atomicOr(&st->err, ERR_MOVERS);
                    b = 0xFFFFFFFFu;
                }
            }
            s_mvbase = b;
        }
        __syncthreads();
        if (moved && s_mvbase != 0xFFFFFFFFu) {
            const uint32_t rank = (uint32_t)__popcll(bal & ((1ull << lane) - 1ull));
            movers[s_mvbase + (w ? s_mv[0] : 0u) + rank] = make_uint2(newkey, i);
        }
    }
}

// Split path, second loop (section 3.4): one lane per compacted contact of
// the tile.  Velocities come through the permutation, history is matched by
// partner id, the contact law runs, and each particle then adds its own
// contacts in row order (ascending partner id, faces last) from LDS.
//
// HK > 0: the contacts come as the adjacency lists of the half search
// (k_detect_half, HK slots per particle) instead of rows.  The workgroup first
// turns its particles' lists into their rows, ordered by partner id, in the
// tile's region of the contact list (what the full search writes), then runs
// as above; the lists' counters are reset, also when the step is abandoned.
template <typename R, int HK = 0>
__global__ __launch_bounds__(TILE) void k_force(
    const double4* __restrict__ xr_x,
    const double2* __restrict__ vw, const uint8_t* __restrict__ mat,
    double4* __restrict__ xr_b, double2* __restrict__ vw_b, uint8_t* __restrict__ mat_b,
    const uint2* __restrict__ rows, const uint32_t* __restrict__ col_j,
    const uint2* __restrict__ rows_old, const uint32_t* __restrict__ perm,
    const uint32_t* __restrict__ tab_pid_old, const double* __restrict__ tab_dt_old,
    uint32_t* __restrict__ tab_pid_new, double* __restrict__ tab_dt_new, uint64_t cap,
    uint2* __restrict__ cells, uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
    R* __restrict__ fo, PoolView P, const Job* __restrict__ jobs, uint32_t* __restrict__ oldkeys,
    uint2* __restrict__ movers, uint32_t* __restrict__ deg, const uint2* __restrict__ adj,
    uint2* __restrict__ rows_out, uint32_t* __restrict__ col_out, uint32_t slots) {
    __shared__ double4 s_x[TILE];
    // the velocities and the chunk's forces; with HK, first the partner ids
    // of the lists (HK slots per particle)
    constexpr size_t VWF = sizeof(double2) * 3 * TILE + sizeof(R) * 6 * TILE;
    // at most 16 list slots per lane are held in LDS: a longer list (only
    // after a row overflow, and rare then) reads its further partner ids
    // from the list itself, so 32 slots need no more LDS than 16
    constexpr uint32_t LK = HK < 16 ? (uint32_t)HK : 16u;
    constexpr size_t LST = (size_t)LK * TILE * 4;
    __shared__ __align__(16) unsigned char s_u[VWF > LST ? VWF : LST];
    double2(*const s_vw)[TILE] = reinterpret_cast<double2(*)[TILE]>(s_u);
    R(*const s_f)[TILE] = reinterpret_cast<R(*)[TILE]>(s_u + sizeof(double2) * 3 * TILE);
    __shared__ uint2 s_old[TILE];
    __shared__ uint32_t s_excl[TILE + 1];
    __shared__ uint8_t s_mat[TILE];
    __shared__ uint32_t s_w[TILE / 64];
    __shared__ uint32_t s_base, s_total, s_flag;
    Status* st = P.st;
    const int t = threadIdx.x;
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
    // with HK the lane's list length and entries and its own state are read
    // before the job lookup, so that they are in flight together; every
    // index is a position (a stale permutation entry is clamped), and lanes
    // outside a running job ignore what they read
    uint32_t d = 0;
    uint2 e0[4];
    double4 xi0 = make_double4(0, 0, 0, 0);
    double2 v0 = make_double2(0, 0), v1 = v0, v2 = v0;
    uint2 orow0 = make_uint2(0, 0);
    uint8_t m80 = 0;
    if (HK) {
        // the list length first, then the loads that do not need it, so
        // that its round trip overlaps theirs
        const uint32_t ip = tile * TILE + t;
        d = deg[ip];
        const uint32_t pq = perm[ip];
        if (d) deg[ip] = 0;
        const uint32_t c0 = d <= (uint32_t)HK ? d : 0u;
#pragma unroll
        for (int m = 0; m < 4; ++m)
            e0[m] = (uint32_t)m < c0 ? adj[(size_t)m * P.ns + ip] : make_uint2(0u, 0u);
        const uint32_t q = pq < P.ns ? pq : ip;
        xi0 = xr_x[q];
        v0 = vw[q];
        v1 = vw[P.ns + q];
        v2 = vw[2 * (size_t)P.ns + q];
        orow0 = rows_old[q];
        m80 = mat ? mat[q] : (uint8_t)0;
    }
    if (skip_if_error(st, &s_flag)) return;

    const uint32_t p0 = tile * TILE;
    const uint32_t ns = P.ns;
    uint32_t jb;
    const Job* Jp = tile_job(jobs, P, tile, jb);
    if (!Jp) {
        idle_tile(P, jobs, tile, jb, t, xr_x, vw, mat, xr_b, vw_b, mat_b, perm, keys, vals, oldkeys,
                  movers != nullptr);
        return;
    }
    const Job& J = *Jp;
    const Geo& G = J.g;
    const MatTable* __restrict__ mt = P.mats + J.mat;
    cells += J.cell_base;
    const uint32_t i = p0 + t;
    const uint32_t n = J.p0 + J.n;  // end of the job's particles
    if (i >= n) {
        // ghost slot after the job's last particle: sorts last, stays in place
        fixed_sort_input(keys, vals, oldkeys, movers != nullptr, i, tile_key_of(P, tile) | P.lmask);
    }
    const uint32_t nt = (n - p0) < (uint32_t)TILE ? (n - p0) : (uint32_t)TILE;
    uint2 row = make_uint2(0, 0);
    uint2 orow = make_uint2(0, 0);
    if (HK) {
        // own state: the velocities stay in registers while the lists are
        // ranked in s_u, the rest goes to its place (a lane of a running job
        // has at most its own list: no list outside one)
        const bool mine = i < n;
        const bool over = mine && d > (uint32_t)HK;
        const uint32_t cnt = (mine && !over) ? d : 0u;
        if (mine) {
            orow = orow0;
            s_x[t] = xi0;
            s_mat[t] = m80;
        }
        if (over) atomicOr(&st->err, ERR_ROW);
        if (__syncthreads_or(over)) return;
        uint32_t tot;
        const uint32_t ex = block_excl_scan<TILE / 64>(cnt, s_w, tot);
        const uint32_t rbase = tile * (uint32_t)TILE * slots;
        if (tot > (uint32_t)TILE * slots) {
            if (t == 0) {
                atomicOr(&st->err, ERR_CAPACITY);
                atomicMax(&st->need, tot);
            }
            return;
        }
        row = make_uint2(rbase + ex, cnt);
        if (mine) rows_out[i] = row;
        if (t == 0) P.ts[tile].m_step = tot;
        // the list's partner ids into the lane's column of s_u; each entry
        // then goes to the place its rank by partner id gives it in the row
        // (ties, which distinct ids never make, by list order)
        uint32_t* const s_lp = reinterpret_cast<uint32_t*>(s_u);
#pragma unroll
        for (int m = 0; m < 4; ++m)
            if ((uint32_t)m < cnt) s_lp[m * TILE + t] = e0[m].y;
        for (uint32_t k = 4; k < cnt && k < LK; ++k) s_lp[k * TILE + t] = adj[(size_t)k * ns + i].y;
        auto place = [&](const uint2 e, uint32_t k) {
            uint32_t rank = 0;
            for (uint32_t m = 0; m < cnt; ++m) {
                const uint32_t pm = (HK <= 16 || m < LK) ? s_lp[m * TILE + t]
                                                         : adj[(size_t)m * ns + i].y;
                rank += (pm < e.y || (pm == e.y && m < k)) ? 1u : 0u;
            }
            col_out[rbase + ex + rank] = e.x;
        };
#pragma unroll
        for (int m = 0; m < 4; ++m)
            if ((uint32_t)m < cnt) place(e0[m], (uint32_t)m);
        for (uint32_t k = 4; k < cnt; ++k) place(adj[(size_t)k * ns + i], k);
        s_excl[t] = ex;
        if (t == 0) s_excl[TILE] = tot;
        __syncthreads();  // s_u turns into the velocities and forces
        if (mine) {
            s_vw[0][t] = v0;
            s_vw[1][t] = v1;
            s_vw[2][t] = v2;
        }
    } else if (i < n) {
        // own records through the permutation
        const uint32_t q = perm[i];
        row = rows[i];
        orow = rows_old[q];
        s_x[t] = xr_x[q];
        s_vw[0][t] = vw[q];
        s_vw[1][t] = vw[ns + q];
        s_vw[2][t] = vw[2 * (size_t)ns + q];
        s_mat[t] = mat ? mat[q] : (uint8_t)0;
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
            const double4 a = s_x[o];
            const int mi = s_mat[o];
            const PairTerms<R> p = pair_terms<R>(G, mt, HK ? col_out[g] : col_j[g], a, s_vw[0][o],
                                                 s_vw[1][o], s_vw[2][o], mi, xr_x, vw, mat, perm,
                                                 ns, J.xw);
            double dtx, dty, dtz;
            matched += history_of<true>(s_old[o], p.pid, tab_pid_old, tab_dt_old, cap, dtx, dty,
                                        dtz) ? 1u : 0u;
            const int pr = mi * MAXMAT + p.mj;
            R F[3], T[3];
            contact_law<R>(p.nx, p.ny, p.nz, p.dn, p.vx, p.vy, p.vz, p.rwx, p.rwy, p.rwz, dtx, dty,
                           dtz, p.rs, p.ms, (R)meta_r(a.w), (R)mt->kn_pref[pr],
                           (R)mt->kt_pref[pr], (R)mt->alpha[pr], (R)mt->mu[pr], G.dt, F, T);
            tab_pid_new[g] = p.pid;
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
    finish_tile<R>(P, G, mt, tile, jb, t, i, n, s_x[t], s_vw[0][t], s_vw[1][t], s_vw[2][t],
                   s_mat[t], acc, true, matched, (i < n) ? orow.y : 0u, nullptr, xr_b, vw_b, mat_b,
                   cells, true, keys, vals, fo, oldkeys, movers);
}

// The split as the paper has it (section 3.4): the second loop runs in the
// particle's own thread over the contacts its first loop found, with no
// compaction across the workgroup, so a wavefront takes as long as its lane
// with the most contacts.  Kept as the comparison for the compacted force
// kernel; the per-contact terms and the summation order are the same.
template <typename R>
__global__ __launch_bounds__(TILE) void k_force_thread(
    const double4* __restrict__ xr_x,
    const double2* __restrict__ vw, const uint8_t* __restrict__ mat,
    double4* __restrict__ xr_b, double2* __restrict__ vw_b, uint8_t* __restrict__ mat_b,
    const uint2* __restrict__ rows, const uint32_t* __restrict__ col_j,
    const uint2* __restrict__ rows_old, const uint32_t* __restrict__ perm,
    const uint32_t* __restrict__ tab_pid_old, const double* __restrict__ tab_dt_old,
    uint32_t* __restrict__ tab_pid_new, double* __restrict__ tab_dt_new, uint64_t cap,
    uint2* __restrict__ cells, uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
    R* __restrict__ fo, PoolView P, const Job* __restrict__ jobs, uint32_t* __restrict__ oldkeys,
    uint2* __restrict__ movers) {
    __shared__ uint32_t s_flag;
    Status* st = P.st;
    if (skip_if_error(st, &s_flag)) return;
    const int t = threadIdx.x;
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t p0 = tile * TILE;
    const uint32_t ns = P.ns;
    uint32_t jb;
    const Job* Jp = tile_job(jobs, P, tile, jb);
    if (!Jp) {
        idle_tile(P, jobs, tile, jb, t, xr_x, vw, mat, xr_b, vw_b, mat_b, perm, keys, vals, oldkeys,
                  movers != nullptr);
        return;
    }
    const Job& J = *Jp;
    const Geo& G = J.g;
    const MatTable* __restrict__ mt = P.mats + J.mat;
    const uint32_t i = p0 + t;
    const uint32_t n = J.p0 + J.n;
    if (i >= n) {
        fixed_sort_input(keys, vals, oldkeys, movers != nullptr, i, tile_key_of(P, tile) | P.lmask);
    }
    R acc[6] = {0, 0, 0, 0, 0, 0};
    uint32_t matched = 0;
    double4 a = make_double4(0.0, 0.0, 0.0, 0.0);
    double2 a0 = make_double2(0.0, 0.0), a1 = a0, a2 = a0;
    int mi = 0;
    uint2 orow = make_uint2(0, 0);
    if (i < n) {
        const uint32_t q = perm[i];
        const uint2 row = rows[i];
        orow = rows_old[q];
        a = xr_x[q];
        a0 = vw[q];
        a1 = vw[ns + q];
        a2 = vw[2 * (size_t)ns + q];
        mi = mat ? mat[q] : 0;
        if ((uint64_t)row.x + row.y > cap) {  // cannot happen after a clean detect
            atomicOr(&st->err, ERR_CAPACITY);
        } else {
            for (uint32_t k = row.x; k < row.x + row.y; ++k) {
                const uint32_t code = col_j[k];
                const PairTerms<R> p = pair_terms<R>(G, mt, code, a, a0, a1, a2, mi, xr_x, vw,
                                                     mat, perm, ns, J.xw);
                double dtx, dty, dtz;
                matched += history_of<true>(orow, p.pid, tab_pid_old, tab_dt_old, cap, dtx, dty,
                                            dtz) ? 1u : 0u;
                const int pr = mi * MAXMAT + p.mj;
                R F[3], T[3];
                contact_law<R>(p.nx, p.ny, p.nz, p.dn, p.vx, p.vy, p.vz, p.rwx, p.rwy, p.rwz, dtx,
                               dty, dtz, p.rs, p.ms, (R)meta_r(a.w), (R)mt->kn_pref[pr],
                               (R)mt->kt_pref[pr], (R)mt->alpha[pr], (R)mt->mu[pr], G.dt, F, T);
                tab_pid_new[k] = p.pid;
                tab_dt_new[k] = dtx;
                tab_dt_new[cap + k] = dty;
                tab_dt_new[2 * cap + k] = dtz;
                acc[0] += F[0];
                acc[1] += F[1];
                acc[2] += F[2];
                acc[3] += T[0];
                acc[4] += T[1];
                acc[5] += T[2];
            }
        }
    }
    finish_tile<R>(P, G, mt, tile, jb, t, i, n, a, a0, a1, a2, mi, acc, true, matched, orow.y,
                   nullptr, xr_b, vw_b, mat_b, cells + J.cell_base, true, keys, vals, fo, oldkeys,
                   movers);
}

// ------------------------------------------------------- action-reaction
// Variant that computes each particle pair once (the scheme section 3.3
// avoids): the particle with the lower id owns the pair.  First kernel: one
// lane per compacted contact of the tile, as in the force kernel, but the
// contact law runs only for owned entries (partner id above the particle's)
// and faces.  The pair force F and n x F go to the entry's slot of `pf` (six
// planes of cap values) for both particles' sums; every entry gets its
// partner id, and the history table keeps the tangential displacement in the
// owner's entry only (zero in the other).  The churn counters count an owned
// pair that carried history twice, as both of its directed contacts did.
template <typename R>
__global__ __launch_bounds__(TILE) void k_pair_force(
    const double4* __restrict__ xr_x, const double2* __restrict__ vw,
    const uint8_t* __restrict__ mat, const uint2* __restrict__ rows,
    const uint32_t* __restrict__ col_j, const uint2* __restrict__ rows_old,
    const uint32_t* __restrict__ perm, const uint32_t* __restrict__ tab_pid_old,
    const double* __restrict__ tab_dt_old, uint32_t* __restrict__ tab_pid_new,
    double* __restrict__ tab_dt_new, uint64_t cap, R* __restrict__ pf, PoolView P,
    const Job* __restrict__ jobs) {
    __shared__ double4 s_x[TILE];
    __shared__ double2 s_vw[3][TILE];
    __shared__ uint2 s_old[TILE];
    __shared__ uint32_t s_excl[TILE + 1];
    __shared__ uint8_t s_mat[TILE];
    __shared__ uint32_t s_base, s_total, s_flag;
    __shared__ uint32_t s_red[4];
    Status* st = P.st;
    if (skip_if_error(st, &s_flag)) return;

    const int t = threadIdx.x;
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t p0 = tile * TILE;
    const uint32_t ns = P.ns;
    uint32_t jb;
    const Job* Jp = tile_job(jobs, P, tile, jb);
    if (!Jp) return;
    const Job& J = *Jp;
    const Geo& G = J.g;
    const MatTable* __restrict__ mt = P.mats + J.mat;
    const uint32_t i = p0 + t;
    const uint32_t n = J.p0 + J.n;
    const uint32_t nt = (n - p0) < (uint32_t)TILE ? (n - p0) : (uint32_t)TILE;
    uint2 row = make_uint2(0, 0);
    uint2 orow = make_uint2(0, 0);
    if (i < n) {
        const uint32_t q = perm[i];
        row = rows[i];
        orow = rows_old[q];
        s_x[t] = xr_x[q];
        s_vw[0][t] = vw[q];
        s_vw[1][t] = vw[ns + q];
        s_vw[2][t] = vw[2 * (size_t)ns + q];
        s_mat[t] = mat ? mat[q] : (uint8_t)0;
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
    uint32_t matched = 0;
    for (uint32_t q = t; q < total; q += TILE) {
        const int o = owner_of(s_excl, q);
        const uint64_t g = (uint64_t)base + q;
        const uint32_t code = col_j[g];
        const double4 a = s_x[o];
        uint32_t pid = code;
        bool own = true;
        if (code < FACE) {
            pid = meta_pid(xr_x[perm[code]].w);
            own = pid > meta_pid(a.w);
        }
        double dtx = 0.0, dty = 0.0, dtz = 0.0;
        R F[3] = {0, 0, 0}, nF[3] = {0, 0, 0};
        if (own) {
            const int mi = s_mat[o];
            const PairTerms<R> p = pair_terms<R>(G, mt, code, a, s_vw[0][o], s_vw[1][o],
                                                 s_vw[2][o], mi, xr_x, vw, mat, perm, ns, J.xw);
            if (history_of<true>(s_old[o], p.pid, tab_pid_old, tab_dt_old, cap, dtx, dty, dtz))
                matched += code < FACE ? 2u : 1u;
            const int pr = mi * MAXMAT + p.mj;
            // with a unit radius the torque output is n x F itself
            contact_law<R>(p.nx, p.ny, p.nz, p.dn, p.vx, p.vy, p.vz, p.rwx, p.rwy, p.rwz, dtx,
                           dty, dtz, p.rs, p.ms, (R)1, (R)mt->kn_pref[pr], (R)mt->kt_pref[pr],
                           (R)mt->alpha[pr], (R)mt->mu[pr], G.dt, F, nF);
        }
        tab_pid_new[g] = pid;
        tab_dt_new[g] = dtx;
        tab_dt_new[cap + g] = dty;
        tab_dt_new[2 * cap + g] = dtz;
        pf[g] = F[0];
        pf[cap + g] = F[1];
        pf[2 * cap + g] = F[2];
        pf[3 * cap + g] = nF[0];
        pf[4 * cap + g] = nF[1];
        pf[5 * cap + g] = nF[2];
    }
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
        P.ts[tile].matched_step = s_red[0] + s_red[2];
        P.ts[tile].old_step = s_red[1] + s_red[3];
    }
}

// Action-reaction variant, second kernel: one lane per particle adds its
// row in order (ascending partner id, faces last): its own entries' F and
// r_i (n x F); for a pair the partner owns, minus the force of the partner's
// entry for this particle (found in the partner's row) and r_i times its
// n x F (the normal and the force both change sign).  Then the end of the
// step as in the force kernel.
template <typename R>
__global__ __launch_bounds__(TILE) void k_ar_sum(
    const double4* __restrict__ xr_x,
    const double2* __restrict__ vw, const uint8_t* __restrict__ mat,
    double4* __restrict__ xr_b, double2* __restrict__ vw_b, uint8_t* __restrict__ mat_b,
    const uint2* __restrict__ rows, const uint32_t* __restrict__ col_j,
    const uint32_t* __restrict__ perm, const uint32_t* __restrict__ tab_pid_new,
    const R* __restrict__ pf, uint64_t cap, uint2* __restrict__ cells,
    uint32_t* __restrict__ keys, uint32_t* __restrict__ vals, R* __restrict__ fo, PoolView P,
    const Job* __restrict__ jobs, uint32_t* __restrict__ oldkeys, uint2* __restrict__ movers) {
    __shared__ uint32_t s_flag;
    Status* st = P.st;
    if (skip_if_error(st, &s_flag)) return;
    const int t = threadIdx.x;
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t p0 = tile * TILE;
    const uint32_t ns = P.ns;
    uint32_t jb;
    const Job* Jp = tile_job(jobs, P, tile, jb);
    if (!Jp) {
        idle_tile(P, jobs, tile, jb, t, xr_x, vw, mat, xr_b, vw_b, mat_b, perm, keys, vals, oldkeys,
                  movers != nullptr);
        return;
    }
    const Job& J = *Jp;
    const Geo& G = J.g;
    const MatTable* __restrict__ mt = P.mats + J.mat;
    const uint32_t i = p0 + t;
    const uint32_t n = J.p0 + J.n;
    if (i >= n) {
        fixed_sort_input(keys, vals, oldkeys, movers != nullptr, i, tile_key_of(P, tile) | P.lmask);
    }
    R acc[6] = {0, 0, 0, 0, 0, 0};
    double4 a = make_double4(0.0, 0.0, 0.0, 0.0);
    double2 a0 = make_double2(0.0, 0.0), a1 = a0, a2 = a0;
    int mi = 0;
    if (i < n) {
        const uint32_t q = perm[i];
        a = xr_x[q];
        a0 = vw[q];
        a1 = vw[ns + q];
        a2 = vw[2 * (size_t)ns + q];
        mi = mat ? mat[q] : 0;
        const R ri = (R)meta_r(a.w);
        const uint32_t pid_i = meta_pid(a.w);
        const uint2 row = rows[i];
        for (uint32_t k = row.x; k < row.x + row.y; ++k) {
            const uint32_t pj = tab_pid_new[k];
            uint64_t g = k;
            R sg = (R)1;
            if (pj < FACE && pj < pid_i) {
                // the partner owns the pair: its entry for this particle (the
                // contact predicate is symmetric, so the partner's row has one)
                const uint2 rj = rows[col_j[k]];
                sg = (R)0;
                for (uint32_t m = rj.x; m < rj.x + rj.y; ++m) {
                    if (col_j[m] == i) {
                        g = m;
                        sg = (R)-1;
                        break;
                    }
                }
            }
            acc[0] += sg * pf[g];
            acc[1] += sg * pf[cap + g];
            acc[2] += sg * pf[2 * cap + g];
            acc[3] += ri * ((sg * sg) * pf[3 * cap + g]);
            acc[4] += ri * ((sg * sg) * pf[4 * cap + g]);
            acc[5] += ri * ((sg * sg) * pf[5 * cap + g]);
        }
    }
    finish_tile<R>(P, G, mt, tile, jb, t, i, n, a, a0, a1, a2, mi, acc, false, 0u, 0u, nullptr,
                   xr_b, vw_b, mat_b, cells + J.cell_base, true, keys, vals, fo, oldkeys, movers);
}

// ------------------------------------------------------------------ fused
// The single loop the paper starts from (section 3.4, Algorithm 1 before the
// split), kept as an ablation of the split path: one lane per particle walks
// its candidates exactly as the detect kernel does and, for every partner it
// touches, matches the history, runs the contact law at once and adds the
// force.  Lanes of a wavefront that find a contact run the contact law while
// the others wait: the divergence the split removes.  The particle's
// contacts go to its own slab of `slots` entries in the tile's region of the
// contact table, in the order they were found (faces last), and the
// per-particle sums follow that order.  Cell bounds are only read here (other
// workgroups may still be walking them); k_clear_cells empties the old ones
// afterwards.
template <typename R, bool PER>
__global__ __launch_bounds__(TILE) void k_fused(
    PoolView P, const Job* __restrict__ jobs, SortedPos xr,
    const float4* __restrict__ xf, const double4* __restrict__ xr_x,
    const double2* __restrict__ vw, const uint8_t* __restrict__ mat, double4* __restrict__ xr_b,
    double2* __restrict__ vw_b, uint8_t* __restrict__ mat_b, uint2* __restrict__ rows,
    uint32_t* __restrict__ col_j, const uint2* __restrict__ rows_old,
    const uint32_t* __restrict__ perm, const uint32_t* __restrict__ tab_pid_old,
    const double* __restrict__ tab_dt_old, uint32_t* __restrict__ tab_pid_new,
    double* __restrict__ tab_dt_new, uint64_t cap, uint32_t slots,
    const uint2* __restrict__ cells, uint32_t* __restrict__ keys, uint32_t* __restrict__ vals,
    R* __restrict__ fo, uint32_t* __restrict__ oldkeys, uint2* __restrict__ movers) {
    static_assert(DTILE == TILE, "the candidate ranges use the detect tile layout");
    constexpr int NWIN = PER ? 18 : 9;
    __shared__ uint2 s_win[(NWIN + 1) * TILE];
    __shared__ uint32_t s_flag;
    Status* st = P.st;
    if (skip_if_error(st, &s_flag)) return;

    const int t = threadIdx.x;
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
    const uint32_t p0 = tile * TILE;
    const uint32_t ns = P.ns;
    uint32_t jb;
    const Job* Jp = tile_job(jobs, P, tile, jb);
    if (!Jp) {
        idle_tile(P, jobs, tile, jb, t, xr_x, vw, mat, xr_b, vw_b, mat_b, perm, keys, vals, oldkeys,
                  movers != nullptr);
        return;
    }
    const Job& J = *Jp;
    const Geo& G = J.g;
    const MatTable* __restrict__ mt = P.mats + J.mat;
    const uint32_t i = p0 + t;
    const uint32_t n = J.p0 + J.n;
    if (i >= n) {
        fixed_sort_input(keys, vals, oldkeys, movers != nullptr, i, tile_key_of(P, tile) | P.lmask);
    }
    R acc[6] = {0, 0, 0, 0, 0, 0};
    uint32_t matched = 0, cnt = 0;
    uint2 orow = make_uint2(0, 0);
    double4 a = make_double4(0.0, 0.0, 0.0, 0.0);
    double2 a0 = make_double2(0.0, 0.0), a1 = a0, a2 = a0;
    int mi = 0;
    const uint64_t slab = ((uint64_t)tile * TILE + (uint64_t)t) * slots;
    if (i < n) {
        const uint32_t q = perm[i];
        orow = rows_old[q];
        a = xr[i];
        a0 = vw[q];
        a1 = vw[ns + q];
        a2 = vw[2 * (size_t)ns + q];
        mi = mat ? mat[q] : 0;
        const double rid = (double)meta_r(a.w);
        const R ri = (R)meta_r(a.w);
        // a contact found: history, contact law and sum at once
        auto contact = [&](uint32_t code) {
            if (cnt < slots) {
                const uint64_t g = slab + cnt;
                const PairTerms<R> p =
                    pair_terms<R>(G, mt, code, a, a0, a1, a2, mi, xr_x, vw, mat, perm, ns, J.xw);
                double dtx, dty, dtz;
                matched += history_of<false>(orow, p.pid, tab_pid_old, tab_dt_old, cap, dtx, dty,
                                             dtz) ? 1u : 0u;
                const int pr = mi * MAXMAT + p.mj;
                R F[3], T[3];
                contact_law<R>(p.nx, p.ny, p.nz, p.dn, p.vx, p.vy, p.vz, p.rwx, p.rwy, p.rwz, dtx,
                               dty, dtz, p.rs, p.ms, ri, (R)mt->kn_pref[pr], (R)mt->kt_pref[pr],
                               (R)mt->alpha[pr], (R)mt->mu[pr], G.dt, F, T);
                acc[0] += F[0];
                acc[1] += F[1];
                acc[2] += F[2];
                acc[3] += T[0];
                acc[4] += T[1];
                acc[5] += T[2];
                col_j[g] = code;
                tab_pid_new[g] = p.pid;
                tab_dt_new[g] = dtx;
                tab_dt_new[(size_t)cap + g] = dty;
                tab_dt_new[2 * (size_t)cap + g] = dtz;
            }
            ++cnt;
        };
        // the exact FP64 predicate on a candidate that passed the pre-filter
        auto touches = [&](uint32_t c) {
            const double4 b = xr[c];
            double dx = b.x - a.x, dy = b.y - a.y, dz = b.z - a.z;
            if (PER) {
                double Sx, Sy, Sz;
                int ky;
                image_shift(G, dx, dy, dz, Sx, Sy, Sz, ky);
                dx = dx + Sx;
                dy = dy + Sy;
                dz = dz + Sz;
            }
            return touching(dx, dy, dz, rid + (double)meta_r(b.w));
        };
        const uint32_t nw = candidate_ranges<PER>(G, a, rid, cells + J.cell_base, s_win + t, TILE);
        const PreFilter<PER> pre(G, a, J.margin);
        constexpr uint32_t NONE = 0xFFFFFFFFu;
        if (nw > 0) {
            // the detect kernel's walk: branch-free over the ranges, a
            // sentinel range at the end, four records in flight
            s_win[nw * TILE + t] = make_uint2(NONE, NONE);
            uint32_t w = 0;
            uint2 rg = s_win[t];
            uint2 rn = s_win[TILE + t];
            uint32_t j = rg.x;
            auto next = [&]() -> uint32_t {
                const uint32_t c = j;
                const bool live = c != NONE;
                const bool sw = live && c + 1 == rg.y;
                j = !live ? NONE : (sw ? rn.x : c + 1);
                rg.y = sw ? rn.y : rg.y;
                w += sw ? 1u : 0u;
                rn = s_win[min(w + 1, nw) * TILE + t];
                return c;
            };
            uint32_t j0 = next(), j1 = next(), j2 = next(), j3 = next();
            float4 q0 = xf[j0 < ns ? j0 : i], q1 = xf[j1 < ns ? j1 : i];
            float4 q2 = xf[j2 < ns ? j2 : i], q3 = xf[j3 < ns ? j3 : i];
#define DEM_FUSED_STEP(Q, JQ)                                       \
    {                                                               \
        if (JQ == NONE) break;                                      \
        if (JQ != i && JQ < ns && pre(Q) && touches(JQ)) contact(JQ); \
        JQ = next();                                                \
        Q = xf[JQ < ns ? JQ : i];                                   \
    }
            for (;;) {
                DEM_FUSED_STEP(q0, j0)
                DEM_FUSED_STEP(q1, j1)
                DEM_FUSED_STEP(q2, j2)
                DEM_FUSED_STEP(q3, j3)
            }
#undef DEM_FUSED_STEP
        }
        if (G.walls) {
            for (int f = 0; f < 6; ++f) {
                if (!(G.walls & (1u << f))) continue;
                const int ax = f >> 1;
                const double pc = ax == 0 ? a.x : (ax == 1 ? a.y : a.z);
                const double dist = (f & 1) ? G.hi[ax] - pc : pc - G.lo[ax];
                if (dist < rid) contact(FACE + (uint32_t)f);
            }
        }
        for (uint32_t k = 0; k < J.nxw; ++k)
            if (wall_touch(J.xw[k], a.x, a.y, a.z, rid)) contact(FACE + 6u + k);
        if (cnt > slots) {
            // the slab is too small: the step is redone with wider slabs
            atomicOr(&st->err, ERR_CAPACITY);
            atomicMax(&st->need, cnt * (uint32_t)TILE);
            cnt = 0;
        }
        rows[i] = make_uint2((uint32_t)slab, cnt);
    }
    finish_tile<R>(P, G, mt, tile, jb, t, i, n, a, a0, a1, a2, mi, acc, true, matched, orow.y, &cnt,
                   xr_b, vw_b, mat_b, nullptr, false, keys, vals, fo, oldkeys, movers);
}

// After the fused kernel: the first particle of each cell of the order the
// step started from empties that cell's bounds (the reorder writes those of
// the new order).
__global__ __launch_bounds__(TILE) void k_clear_cells(PoolView P, const Job* __restrict__ jobs,
                                                      SortedPos xr,
                                                      uint2* __restrict__ cells) {
    __shared__ uint32_t s_flag;
    if (skip_if_error(P.st, &s_flag)) return;
    const uint32_t tile = xcd_tile(blockIdx.x, gridDim.x);
    uint32_t jb;
    const Job* Jp = tile_job(jobs, P, tile, jb);
    if (!Jp) return;
    const Geo& G = Jp->g;
    const uint32_t i = tile * TILE + threadIdx.x;
    if (i >= Jp->p0 + Jp->n) return;
    const double4 a = xr[i];
    uint2* c = cells + Jp->cell_base;
    const uint32_t lin = key_lin(G, cell_key(G, a.x, a.y, a.z));
    if (c[lin].x == i) c[lin] = make_uint2(0, 0);
}

// End of a step for one job: time, step count and shear offsets advance; a
// job that produced a non-finite state is marked failed.
// The descriptors are double-buffered: the kernels of a step read `in`, and
// the end of the step writes every descriptor, advanced or copied, to `out`,
// which the next step reads.  So the end of a step can run before the
// step's last kernels (which still read `in`), and a step abandoned at any
// point leaves the descriptors it started from intact.
__device__ inline void tick_job(const Job* __restrict__ in, Job* __restrict__ out,
                                const uint32_t* __restrict__ job_fail, uint32_t k) {
    Job J = in[k];
    if (J.status == JOB_ACTIVE) {
        if (job_fail[k]) {
            J.status = JOB_FAILED;
        } else {
            const double t = J.t + J.g.dt;
            J.t = t;
            if (J.g.le) {
                J.g.le_shift = fmod(J.g.le_dv * t, J.g.L[0]);
                J.g.le_shift_next = fmod(J.g.le_dv * (t + J.g.dt), J.g.L[0]);
            }
            J.steps_done += 1;
            if (J.steps_left != 0xFFFFFFFFu && --J.steps_left == 0) J.status = JOB_DONE;
        }
    }
    out[k] = J;
}

// ------------------------------------------------------------ merge sort
// Between two steps few particles change cell.  The others keep their key
// and are still in key order, so the stable order of the step is the merge
// of that sequence with the movers sorted by (new key, position), which is
// exactly what the radix sort produces.  A position p before the step has
// key oldkeys[p], and (oldkeys[p], p) increases with p.
//
// k_mov_sort: one workgroup sorts the movers by (key, position) and by
// position (bitonic networks in LDS); k_place then places every particle.
__global__ __launch_bounds__(1024) void k_mov_sort(const uint2* __restrict__ movers,
                                                   unsigned long long* __restrict__ mk,
                                                   uint32_t* __restrict__ mp, const Status* st,
                                                   const Job* __restrict__ jin,
                                                   Job* __restrict__ jout,
                                                   const uint32_t* __restrict__ job_fail,
                                                   uint32_t njobs) {
    // both orders at once: (key, position) in s_k, position in s_p, each
    // compare-exchange stage of the bitonic network applied to both arrays
    __shared__ unsigned long long s_k[MAX_MOVERS];
    __shared__ uint32_t s_p[MAX_MOVERS];
    __shared__ uint32_t s_flag;
    const int t = threadIdx.x;
    // the count and the first movers are read before the error check
    const uint32_t M = ((ConstPtr<Status>)st)->movers;
    const uint2 e0 = movers[t];  // t < 1024 <= MAX_MOVERS
    if (skip_if_error(st, &s_flag)) return;
    // the end of the step for every job (its force kernel has run)
    for (uint32_t k = (uint32_t)t; k < njobs; k += 1024) tick_job(jin, jout, job_fail, k);
    if (M == 0) return;
    if (M <= 64) {
        // few movers (the common case): the first wavefront sorts both
        // orders in registers, one mover per lane, with the same bitonic
        // network across lanes (lane t and lane t ^ j compare-exchange;
        // the lower lane keeps the minimum in an ascending block)
        if (t >= 64) return;
        unsigned long long k = (uint32_t)t < M ? ((unsigned long long)e0.x << 32) | e0.y : ~0ull;
        uint32_t p = (uint32_t)t < M ? e0.y : 0xFFFFFFFFu;
        for (int kk = 2; kk <= 64; kk <<= 1) {
            for (int j = kk >> 1; j > 0; j >>= 1) {
                const uint32_t klo = __shfl_xor((uint32_t)k, j, 64);
                const uint32_t khi = __shfl_xor((uint32_t)(k >> 32), j, 64);
                const unsigned long long ko = ((unsigned long long)khi << 32) | klo;
                const uint32_t po = __shfl_xor(p, j, 64);
                const bool keep_min = ((t & j) == 0) == ((t & kk) == 0);
                k = keep_min ? (ko < k ? ko : k) : (ko > k ? ko : k);
                p = keep_min ? (po < p ? po : p) : (po > p ? po : p);
            }
        }
        if ((uint32_t)t < M) {
            mk[t] = k;
            mp[t] = p;
        }
        return;
    }
    uint32_t n2 = 1;
    while (n2 < M) n2 <<= 1;
    for (uint32_t q = t; q < n2; q += 1024) {
        if (q < M) {
            const uint2 e = q == (uint32_t)t ? e0 : movers[q];
            s_k[q] = ((unsigned long long)e.x << 32) | e.y;
            s_p[q] = e.y;
        } else {
            s_k[q] = ~0ull;
            s_p[q] = 0xFFFFFFFFu;
        }
    }
    __syncthreads();
    const uint32_t half = n2 / 2;
    for (uint32_t k = 2; k <= n2; k <<= 1) {
        for (uint32_t jj = k >> 1; jj > 0; jj >>= 1) {
            // items [0, half) exchange in s_k, [half, n2) in s_p
            for (uint32_t w = t; w < n2; w += 1024) {
                const uint32_t q = w < half ? w : w - half;
                const uint32_t lo = 2 * q - (q & (jj - 1));
                const uint32_t hi = lo + jj;
                const bool up = (lo & k) == 0;
                if (w < half) {
                    const unsigned long long u = s_k[lo], v = s_k[hi];
                    if ((u > v) == up) {
                        s_k[lo] = v;
                        s_k[hi] = u;
                    }
                } else {
                    const uint32_t u = s_p[lo], v = s_p[hi];
                    if ((u > v) == up) {
                        s_p[lo] = v;
                        s_p[hi] = u;
                    }
                }
            }
            __syncthreads();
        }
    }
    for (uint32_t q = t; q < M; q += 1024) {
        mk[q] = s_k[q];
        mp[q] = s_p[q];
    }
}

// Number of entries of the sorted a[0, m) below v.
template <typename T>
__device__ inline uint32_t count_below(const T* __restrict__ a, uint32_t m, T v) {
    uint32_t lo = 0, hi = m;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// k_place: one workgroup per tile of positions.  Every unchanged particle
// moves by the movers that leave before it and the movers that arrive before
// it; both counts are found once per tile and are the same for the whole
// tile unless a mover leaves from or arrives inside it.  The movers whose
// (key, position) falls between this tile's first old (key, position) and
// the next tile's are placed by this tile (the first tile also takes those
// that sort before every position): the unchanged particles before a
// mover are the positions before it in old order (all positions before the
// tile, and those of the tile found by binary search) less the movers among
// them.  Mover lists of up to LDS_MOVERS entries are searched in LDS.
constexpr uint32_t LDS_MOVERS = 512;

template <typename K>
__device__ inline uint32_t count_below_in(const K* lds, const K* glob, bool in_lds, uint32_t m,
                                          K v) {
    return in_lds ? count_below(lds, m, v) : count_below(glob, m, v);
}

__global__ __launch_bounds__(TILE) void k_place(PoolView P, const Job* __restrict__ jobs,
                                                const uint32_t* __restrict__ oldkeys,
                                                const unsigned long long* __restrict__ mk,
                                                const uint32_t* __restrict__ mp,
                                                uint32_t* __restrict__ keys_s,
                                                const double4* __restrict__ xr_y,
                                                float4* __restrict__ xf,
                                                uint32_t* __restrict__ perm,
                                                uint2* __restrict__ cells) {
    __shared__ unsigned long long s_mk[LDS_MOVERS];
    __shared__ uint32_t s_mp[LDS_MOVERS];
    __shared__ unsigned long long s_ok[TILE];
    __shared__ uint32_t s_c[4];
    __shared__ uint32_t s_flag;
    // the mover count, the lane's key and its new state's position are read
    // before the error check, so that they are in flight together
    const uint32_t M = ((ConstPtr<Status>)P.st)->movers;
    const int t = threadIdx.x;
    const uint32_t N = P.ntiles * TILE;
    const uint32_t p0 = blockIdx.x * TILE, i = p0 + t;
    const uint32_t ok = oldkeys[i];
    const double4 pi = xr_y[i];
    if (skip_if_error(P.st, &s_flag)) return;
    auto key_of = [](uint32_t k, uint32_t p) { return ((unsigned long long)k << 32) | p; };
    // the new order's sorted key, and for a particle of a running job its
    // FP32 record and source position, at `dest`
    auto emit = [&](uint32_t dest, uint32_t key, uint32_t src, const double4& q, const Job* J) {
        keys_s[dest] = key;
        if (J) {
            xf[dest] = far_record(J->g, q);
            perm[dest] = src;
        }
    };
    uint32_t jb;
    const Job* Jt = tile_job(jobs, P, blockIdx.x, jb);
    // a lane's own particle: in a running job, or in a finished one (whose
    // positions map to themselves)
    const Job* Ji = Jt && i < Jt->p0 + Jt->n ? Jt : nullptr;
    if (!Jt && jb != NO_JOB && i < ((ConstPtr<Job>)jobs)[jb].p0 + ((ConstPtr<Job>)jobs)[jb].n)
        perm[i] = i;
    if (M == 0) {
        emit(i, ok, i, pi, Ji);
        return;
    }
    const bool in_lds = M <= LDS_MOVERS;
    if (in_lds) {
        for (uint32_t q = t; q < M; q += TILE) {
            s_mk[q] = mk[q];
            s_mp[q] = mp[q];
        }
    }
    s_ok[t] = key_of(ok, i);
    __syncthreads();
    if (t < 4) {
        // movers leaving before the tile / before the next tile; movers whose
        // place is before the tile's first / the next tile's first position
        uint32_t c;
        if (t == 0) c = count_below_in(s_mp, mp, in_lds, M, p0);
        else if (t == 1) c = count_below_in(s_mp, mp, in_lds, M, p0 + TILE);
        else if (t == 2) c = count_below_in(s_mk, mk, in_lds, M, s_ok[0]);
        else c = p0 + TILE < N ? count_below_in(s_mk, mk, in_lds, M,
                                                key_of(oldkeys[p0 + TILE], p0 + TILE))
                               : M;
        s_c[t] = c;
    }
    __syncthreads();
    // a position is a mover's if the sorted mover positions hold it (none
    // of the tile's unless movers leave from inside it)
    uint32_t leave = s_c[0];
    bool moved = false;
    if (s_c[1] != s_c[0]) {
        leave = count_below_in(s_mp, mp, in_lds, M, i);
        moved = leave < M && (in_lds ? s_mp[leave] : mp[leave]) == i;
    }
    if (!moved) {
        uint32_t arrive = s_c[2];
        if (s_c[3] != s_c[2]) arrive = count_below_in(s_mk, mk, in_lds, M, key_of(ok, i));
        const uint32_t dest = i - leave + arrive;
        if (dest >= N)  // inconsistent input: redo the step with the radix sort
            atomicOr(&P.st->err, ERR_MOVERS);
        else
            emit(dest, ok, i, pi, Ji);
    }
    // the first tile also places the movers that sort before every position
    const uint32_t mlo = blockIdx.x == 0 ? 0u : s_c[2];
    for (uint32_t m = mlo + t; m < s_c[3]; m += TILE) {
        const unsigned long long e = in_lds ? s_mk[m] : mk[m];
        const uint32_t lb = p0 + count_below(s_ok, (uint32_t)TILE, e);
        const uint32_t dest = lb - count_below_in(s_mp, mp, in_lds, M, lb) + m;
        const uint32_t pos = (uint32_t)e;
        if (dest >= N || pos >= N) {
            atomicOr(&P.st->err, ERR_MOVERS);
            continue;
        }
        uint32_t jm;
        const Job* J = tile_job(jobs, P, pos / TILE, jm);
        emit(dest, (uint32_t)(e >> 32), pos, xr_y[pos], J);
        // the mover's old cell may be left empty: its bounds are emptied
        // here, and the bounds kernel writes those of every cell the new
        // order fills (the search of this step has read them already)
        if (J) cells[J->cell_base + key_lin(J->g, oldkeys[pos] & P.lmask)] = make_uint2(0, 0);
    }
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

// One workgroup per REORDER_TILES tiles.  The new sorted order: with GATHER
// (after the radix sort) the permutation into the buffer just written, the
// FP32 records made from it (a finished job's positions map to themselves);
// in every case the cell bounds and the step's counters.  The merge sort's
// placement writes the permutation and records itself (k_place).  Positions
// of free tiles and ghost slots kept their place in the sort and are left
// alone.
constexpr uint32_t REORDER_TILES = 2;
template <bool GATHER>
__global__ __launch_bounds__(TILE) void k_reorder(PoolView P, const Job* __restrict__ jobs,
                                                  const uint32_t* __restrict__ keys_s,
                                                  const uint32_t* __restrict__ vals_s,
                                                  const double4* __restrict__ xr_y,
                                                  float4* __restrict__ xf,
                                                  uint32_t* __restrict__ perm,
                                                  uint2* __restrict__ cells) {
    __shared__ uint32_t s_flag;
    // REORDER_TILES tiles per workgroup, one position of each per lane: half
    // the wavefronts, so that the whole grid is resident at once
    constexpr uint32_t RT = REORDER_TILES;
    const uint32_t t0 = blockIdx.x * RT;
    // the sorted keys and source indices, the gathered positions and the
    // neighbours' keys are read before the error check and the job lookups,
    // so that all are in flight together (every index is a position; a lane
    // outside a running job ignores what it read)
    uint32_t key[RT], src[RT], key_lo[RT], key_hi[RT];
    double4 p[RT];
#pragma unroll
    for (uint32_t r = 0; r < RT; ++r) {
        const uint32_t i = (t0 + r) * TILE + threadIdx.x;
        key[r] = key_lo[r] = key_hi[r] = 0u;
        src[r] = i;
        p[r] = make_double4(0, 0, 0, 0);
        if (t0 + r < P.ntiles) {
            key[r] = keys_s[i];
            if (GATHER) {
                src[r] = vals_s[i] < P.ns ? vals_s[i] : i;
                p[r] = xr_y[src[r]];
            }
            key_lo[r] = i > 0 ? keys_s[i - 1] : 0u;
            key_hi[r] = i + 1 < P.ns ? keys_s[i + 1] : 0u;
        }
    }
    if (skip_if_error(P.st, &s_flag)) return;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        // the step completes: it counts, and the next one's cell changes
        // start from zero
        P.st->steps_done += 1;
        P.st->movers = 0;
    }
#pragma unroll
    for (uint32_t r = 0; r < RT; ++r) {
        const uint32_t tile = t0 + r;
        if (tile >= P.ntiles) break;
        const uint32_t i = tile * TILE + threadIdx.x;
        uint32_t jb;
        const Job* Jp = tile_job(jobs, P, tile, jb);
        if (!Jp) {
            if (GATHER && jb != NO_JOB && i < jobs[jb].p0 + jobs[jb].n) perm[i] = i;
            continue;
        }
        const Job& J = *Jp;
        const Geo& G = J.g;
        if (threadIdx.x == 0) {
            // the step completed: its counters join the sums
            TileStats& q = P.ts[tile];
            q.m += q.m_step;
            q.matched += q.matched_step;
            q.old += q.old_step;
        }
        const uint32_t end = J.p0 + J.n;
        if (i >= end) continue;
        // a source index is a position by construction; checked (above) so
        // that a sort defect can never read outside the arrays
        if (GATHER) {
            xf[i] = far_record(G, p[r]);
            perm[i] = src[r];
        }
        const uint32_t lin = J.cell_base + key_lin(G, key[r] & P.lmask);
        if (i == J.p0 || key_lo[r] != key[r]) cells[lin].x = i;
        if (i == end - 1 || key_hi[r] != key[r]) cells[lin].y = i + 1;
    }
}

// Cell bounds of the current sorted order, from its positions: after
// a step that was abandoned once the force kernel had started (it empties the
// bounds of the cells it leaves), before that step is redone.
__global__ __launch_bounds__(TILE) void k_rebuild_cells(PoolView P, const Job* __restrict__ jobs,
                                                        SortedPos xs,
                                                        uint2* __restrict__ cells) {
    const uint32_t tile = blockIdx.x;
    uint32_t jb;
    const Job* Jp = tile_job(jobs, P, tile, jb);
    if (!Jp) return;
    const Job& J = *Jp;
    const Geo& G = J.g;
    const uint32_t i = tile * TILE + threadIdx.x;
    const uint32_t end = J.p0 + J.n;
    if (i >= end) return;
    auto key_at = [&](uint32_t q) {
        const double4 p = xs[q];
        return cell_key(G, p.x, p.y, p.z);
    };
    const uint32_t key = key_at(i);
    const uint32_t lin = J.cell_base + key_lin(G, key);
    if (i == J.p0 || key_at(i - 1) != key) cells[lin].x = i;
    if (i == end - 1 || key_at(i + 1) != key) cells[lin].y = i + 1;
}

// New radii for the positions [p0, p0 + n) of one job (rnew indexed by the
// particle id in the meta word): the radius half of the meta word of the
// state buffer the next step reads, of its sorted records, and the radius of
// the FP32 records of the contact search.
__global__ __launch_bounds__(TILE) void k_set_radii(uint32_t p0, uint32_t n,
                                                    const float* __restrict__ rnew,
                                                    double4* __restrict__ xr,
                                                    const uint32_t* __restrict__ perm,
                                                    float4* __restrict__ xf) {
    const uint32_t q = blockIdx.x * TILE + threadIdx.x;
    if (q >= n) return;
    const uint32_t i = p0 + q;
    auto r_of = [&](double w) { return meta_pid(w) < n ? rnew[meta_pid(w)] : meta_r(w); };
    // the sorted record at i: its particle id, which this kernel leaves as
    // it is, is read through the permutation before any record changes
    const uint32_t s = perm[i];
    const float rs = r_of(xr[s < p0 + n && s >= p0 ? s : i].w);
    double4 a = xr[i];
    a.w = __longlong_as_double((long long)pack_meta(r_of(a.w), meta_pid(a.w)));
    xr[i] = a;
    float4 f = xf[i];
    f.w = rs;
    xf[i] = f;
}

// The step's count and the reset of its cell changes when no tile is in use
// (the bounds kernel does both otherwise).
__global__ void k_step_count(PoolView P) {
    if (((ConstPtr<Status>)P.st)->err) return;
    P.st->steps_done += 1;
    P.st->movers = 0;
}

// End of a step: every running job advances (one thread per job).
__global__ void k_tick(PoolView P, const Job* __restrict__ in, Job* __restrict__ out,
                       uint32_t njobs) {
    if (((ConstPtr<Status>)P.st)->err) return;
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < njobs) tick_job(in, out, P.job_fail, k);
}

// ------------------------------------------------------------------ launch
// The pre-filter compares float distances of positions within 3 box lengths
// of the corner: every float coordinate, difference, image shift and sum is
// off by at most a few 2^-24 of 3 L, so 48 such units plus 2^-20 of the
// largest contact distance bound the error of the float distance with a wide
// safety factor.
float detect_margin(const Geo& G) {
    const double Lm = std::max(G.L[0], std::max(G.L[1], G.L[2]));
    const double dmax = 2.0 / std::min(G.inv_cell[0], std::min(G.inv_cell[1], G.inv_cell[2]));
    return (float)(48.0 * 3.0 * Lm * 0x1p-24 + dmax * 0x1p-20);
}

void launch_detect(const PoolView& P, int kmax, const Sorted& S, const uint2* cells, uint2* rows,
                   uint32_t* col_j, uint32_t slots, hipStream_t s) {
    if (P.ntiles == 0) return;
    const uint32_t nb = P.ntiles;
#define DEM_DETECT(K, PER)                                                                        \
    hipLaunchKernelGGL((k_detect<K, PER>), dim3(nb), dim3(DTILE), 0, s, P, P.jobs,               \
                       SortedPos{S.xr, S.perm, P.ns}, S.xf,                                            \
                       cells, rows, col_j, slots)
    const bool per = P.any_periodic;
    if (kmax <= 8) {
        if (per) DEM_DETECT(8, true); else DEM_DETECT(8, false);
    } else if (kmax <= 16) {
        if (per) DEM_DETECT(16, true); else DEM_DETECT(16, false);
    } else {
        if (per) DEM_DETECT(32, true); else DEM_DETECT(32, false);
    }
#undef DEM_DETECT
}

void launch_force(const PoolView& P, bool fp64, const Sorted& S, const State& X, const State& Y,
                  const uint2* rows, const uint32_t* col_j, const uint2* rows_old,
                  const uint32_t* perm, const uint32_t* tab_pid_old, const double* tab_dt_old,
                  uint32_t* tab_pid_new, double* tab_dt_new, uint64_t cap, uint2* cells,
                  uint32_t* keys, uint32_t* vals, void* fo, uint32_t* oldkeys, uint2* movers,
                  hipStream_t s) {
    if (P.ntiles == 0) return;
    const uint32_t nb = P.ntiles;
    if (fp64)
        hipLaunchKernelGGL(k_force<double>, dim3(nb), dim3(TILE), 0, s, X.xr, X.vw, X.mat,
                           Y.xr, Y.vw, Y.mat, rows, col_j, rows_old, perm, tab_pid_old, tab_dt_old,
                           tab_pid_new, tab_dt_new, cap, cells, keys, vals, (double*)fo, P, P.jobs,
                           oldkeys, movers, nullptr, nullptr, nullptr, nullptr, 0u);
    else
        hipLaunchKernelGGL(k_force<float>, dim3(nb), dim3(TILE), 0, s, X.xr, X.vw, X.mat,
                           Y.xr, Y.vw, Y.mat, rows, col_j, rows_old, perm, tab_pid_old, tab_dt_old,
                           tab_pid_new, tab_dt_new, cap, cells, keys, vals, (float*)fo, P, P.jobs,
                           oldkeys, movers, nullptr, nullptr, nullptr, nullptr, 0u);
}

void launch_force_half(const PoolView& P, bool fp64, int kmax, const Sorted& S, const State& X,
                       const State& Y, uint32_t* deg, const uint2* adj, uint2* rows,
                       uint32_t* col_j, uint32_t slots, const uint2* rows_old,
                       const uint32_t* perm, const uint32_t* tab_pid_old,
                       const double* tab_dt_old, uint32_t* tab_pid_new, double* tab_dt_new,
                       uint64_t cap, uint2* cells, uint32_t* keys, uint32_t* vals, void* fo,
                       uint32_t* oldkeys, uint2* movers, hipStream_t s) {
    if (P.ntiles == 0) return;
    const uint32_t nb = P.ntiles;
#define DEM_FORCE_HALF(R, K)                                                                      \
    hipLaunchKernelGGL((k_force<R, K>), dim3(nb), dim3(TILE), 0, s, X.xr, X.vw, X.mat, Y.xr,       \
                       Y.vw, Y.mat, nullptr, nullptr, rows_old, perm, tab_pid_old, tab_dt_old,    \
                       tab_pid_new, tab_dt_new, cap, cells, keys, vals, (R*)fo, P, P.jobs,        \
                       oldkeys, movers, deg, adj, rows, col_j, slots)
    if (fp64) {
        if (kmax <= 8) DEM_FORCE_HALF(double, 8);
        else if (kmax <= 16) DEM_FORCE_HALF(double, 16);
        else DEM_FORCE_HALF(double, 32);
    } else {
        if (kmax <= 8) DEM_FORCE_HALF(float, 8);
        else if (kmax <= 16) DEM_FORCE_HALF(float, 16);
        else DEM_FORCE_HALF(float, 32);
    }
#undef DEM_FORCE_HALF
}

void launch_fused(const PoolView& P, bool fp64, const Sorted& S, const State& X, const State& Y,
                  uint2* rows, uint32_t* col_j, const uint2* rows_old, const uint32_t* perm,
                  const uint32_t* tab_pid_old, const double* tab_dt_old, uint32_t* tab_pid_new,
                  double* tab_dt_new, uint64_t cap, uint32_t slots, uint2* cells, uint32_t* keys,
                  uint32_t* vals, void* fo, uint32_t* oldkeys, uint2* movers, hipStream_t s) {
    if (P.ntiles == 0) return;
    const uint32_t nb = P.ntiles;
#define DEM_FUSED(R, PER)                                                                          \
    hipLaunchKernelGGL((k_fused<R, PER>), dim3(nb), dim3(TILE), 0, s, P, P.jobs,                 \
                       SortedPos{S.xr, S.perm, P.ns}, S.xf, X.xr,                                      \
                       X.vw, X.mat, Y.xr, Y.vw, Y.mat, rows, col_j, rows_old, perm, tab_pid_old,  \
                       tab_dt_old, tab_pid_new, tab_dt_new, cap, slots, cells, keys, vals,        \
                       (R*)fo, oldkeys, movers)
    const bool per = P.any_periodic;
    if (fp64) {
        if (per) DEM_FUSED(double, true); else DEM_FUSED(double, false);
    } else {
        if (per) DEM_FUSED(float, true); else DEM_FUSED(float, false);
    }
#undef DEM_FUSED
    hipLaunchKernelGGL(k_clear_cells, dim3(nb), dim3(TILE), 0, s, P, P.jobs,
                       SortedPos{S.xr, S.perm, P.ns}, cells);
}

void launch_action_reaction(const PoolView& P, bool fp64, const Sorted& S, const State& X,
                            const State& Y, const uint2* rows, const uint32_t* col_j,
                            const uint2* rows_old, const uint32_t* perm,
                            const uint32_t* tab_pid_old, const double* tab_dt_old,
                            uint32_t* tab_pid_new, double* tab_dt_new, uint64_t cap, void* pf,
                            uint2* cells, uint32_t* keys, uint32_t* vals, void* fo,
                            uint32_t* oldkeys, uint2* movers, hipStream_t s) {
    if (P.ntiles == 0) return;
    const uint32_t nb = P.ntiles;
#define DEM_AR(R)                                                                                  \
    hipLaunchKernelGGL(k_pair_force<R>, dim3(nb), dim3(TILE), 0, s, X.xr, X.vw, X.mat, rows,      \
                       col_j, rows_old, perm, tab_pid_old, tab_dt_old, tab_pid_new, tab_dt_new,   \
                       cap, (R*)pf, P, P.jobs);                                                   \
    hipLaunchKernelGGL(k_ar_sum<R>, dim3(nb), dim3(TILE), 0, s, X.xr, X.vw, X.mat, Y.xr,          \
                       Y.vw, Y.mat, rows, col_j, perm, tab_pid_new, (const R*)pf, cap, cells,     \
                       keys, vals, (R*)fo, P, P.jobs, oldkeys, movers)
    if (fp64) {
        DEM_AR(double);
    } else {
        DEM_AR(float);
    }
#undef DEM_AR
}

void launch_force_thread(const PoolView& P, bool fp64, const Sorted& S, const State& X,
                         const State& Y, const uint2* rows, const uint32_t* col_j,
                         const uint2* rows_old, const uint32_t* perm, const uint32_t* tab_pid_old,
                         const double* tab_dt_old, uint32_t* tab_pid_new, double* tab_dt_new,
                         uint64_t cap, uint2* cells, uint32_t* keys, uint32_t* vals, void* fo,
                         uint32_t* oldkeys, uint2* movers, hipStream_t s) {
    if (P.ntiles == 0) return;
    const uint32_t nb = P.ntiles;
    if (fp64)
        hipLaunchKernelGGL(k_force_thread<double>, dim3(nb), dim3(TILE), 0, s, X.xr, X.vw,
                           X.mat, Y.xr, Y.vw, Y.mat, rows, col_j, rows_old, perm, tab_pid_old,
                           tab_dt_old, tab_pid_new, tab_dt_new, cap, cells, keys, vals, (double*)fo,
                           P, P.jobs, oldkeys, movers);
    else
        hipLaunchKernelGGL(k_force_thread<float>, dim3(nb), dim3(TILE), 0, s, X.xr, X.vw,
                           X.mat, Y.xr, Y.vw, Y.mat, rows, col_j, rows_old, perm, tab_pid_old,
                           tab_dt_old, tab_pid_new, tab_dt_new, cap, cells, keys, vals, (float*)fo,
                           P, P.jobs, oldkeys, movers);
}

void launch_detect_half(const PoolView& P, int kmax, const Sorted& S, const uint2* cells,
                        uint32_t* deg, uint2* adj, hipStream_t s) {
    if (P.ntiles == 0) return;
    const uint32_t nb = P.ntiles;
#define DEM_HALF(K, PER)                                                                           \
    hipLaunchKernelGGL((k_detect_half<K, PER>), dim3(nb), dim3(DTILE), 0, s, P, P.jobs,          \
                       SortedPos{S.xr, S.perm, P.ns}, S.xf, cells, deg, adj)
    const bool per = P.any_periodic;
    if (kmax <= 8) {
        if (per) { DEM_HALF(8, true); } else { DEM_HALF(8, false); }
    } else if (kmax <= 16) {
        if (per) { DEM_HALF(16, true); } else { DEM_HALF(16, false); }
    } else {
        if (per) { DEM_HALF(32, true); } else { DEM_HALF(32, false); }
    }
#undef DEM_HALF
}

void launch_merge_sort(const PoolView& P, const uint32_t* oldkeys, const uint2* movers,
                       unsigned long long* mk, uint32_t* mp, uint32_t* keys_s, const State& Y,
                       const Sorted& S, uint32_t* perm, uint2* cells, Job* jobs_next,
                       uint32_t njobs, hipStream_t s) {
    hipLaunchKernelGGL(k_mov_sort, dim3(1), dim3(1024), 0, s, movers, mk, mp, P.st, P.jobs,
                       jobs_next, P.job_fail, njobs);
    if (P.ntiles == 0) return;
    hipLaunchKernelGGL(k_place, dim3(P.ntiles), dim3(TILE), 0, s, P, P.jobs, oldkeys, mk, mp,
                       keys_s, Y.xr, S.xf, perm, cells);
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

void launch_set_radii(uint32_t p0, uint32_t n, const float* rnew, const State& X, const Sorted& S,
                      hipStream_t s) {
    if (n > 0)
        hipLaunchKernelGGL(k_set_radii, dim3((n + TILE - 1) / TILE), dim3(TILE), 0, s, p0, n, rnew,
                           X.xr, S.perm, S.xf);
}

void launch_rebuild_cells(const PoolView& P, const Sorted& S, uint2* cells, hipStream_t s) {
    if (P.ntiles > 0)
        hipLaunchKernelGGL(k_rebuild_cells, dim3(P.ntiles), dim3(TILE), 0, s, P, P.jobs,
                           SortedPos{S.xr, S.perm, P.ns},
                           cells);
}

void launch_reorder(const PoolView& P, Job* jobs_next, uint32_t njobs, bool gather,
                    const uint32_t* keys_s, const uint32_t* vals_s, const State& Y,
                    const Sorted& S, uint32_t* perm, uint2* cells, hipStream_t s) {
    if (P.ntiles == 0) hipLaunchKernelGGL(k_step_count, dim3(1), dim3(1), 0, s, P);
    if (P.ntiles > 0) {
        const uint32_t nwg = (P.ntiles + REORDER_TILES - 1) / REORDER_TILES;
        if (gather)
            hipLaunchKernelGGL(k_reorder<true>, dim3(nwg), dim3(TILE), 0, s, P, P.jobs,
                               keys_s, vals_s, Y.xr, S.xf, perm, cells);
        else
            hipLaunchKernelGGL(k_reorder<false>, dim3(nwg), dim3(TILE), 0, s, P, P.jobs,
                               keys_s, vals_s, Y.xr, S.xf, perm, cells);
    }
    // after the merge sort the step has ended already (k_mov_sort)
    if (gather) {
        const uint32_t nb = (njobs + 255) / 256;
        hipLaunchKernelGGL(k_tick, dim3(nb ? nb : 1), dim3(256), 0, s, P, P.jobs, jobs_next,
                           njobs);
    }
}


double le_offset(const Geo& G, double t) { return G.le ? std::fmod(G.le_dv * t, G.L[0]) : 0.0; }

}  // namespace dem
