// art_device.h -- device-side building blocks of the ART sweep for gfx950:
// HEALPix nested ray directions, the per-ray geometry of Sec. 2.1 (split
// radius, domain exit), and the cell-by-cell march (Amanatides-Woo traversal)
// with optical-depth bookkeeping.
//
// Precision: ray geometry, the running optical depth tau and every decision
// (split / exit / termination) are FP64, so the ray tree does not depend on the
// FP32 rounding of the deposits.  Compiled with -ffp-contract=off.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/art.h"

namespace art {

constexpr int kWave = 64;
constexpr uint32_t kNoChild = 0xffffffffu;

// How a ray's march ended (Sec. 2.1): at the split radius, at the domain
// boundary, or because every bin became optically thick (tau > tau_term).
enum End : int { kExit = 0, kSplit = 1, kTerm = 2 };

// Device status bits (first error wins when reported).
enum Status : uint32_t {
    kStOverflow = 1u,
    kStOutside = 2u,
    kStStuck = 4u,
    kStBadField = 8u,  // a cell with n_H < 0 or non-finite, or x_n outside [0, 1]
};

// Per-call constants of the sweep, passed by value to every kernel.
struct Geo {
    int nx, ny, nz;
    int level0, level_max, n_bins;
    double tau_term, s_H, s_d;
    const double* rot;            // device [9], row-major rotation of the HEALPix directions
    double rmax[ART_MAX_LEVELS];  // r_max(l) = sqrt(3/(pi m_ray)) 2^l
};

// ---------------------------------------------------------------------------
// HEALPix nested scheme (Gorski et al. 2005).
// ---------------------------------------------------------------------------

// Gather the even-position bits of v into the low half (inverse of the
// Z-order interleave used by the nested numbering inside a base face).
__device__ __forceinline__ uint32_t gather_even_bits(uint64_t v) {
    v &= 0x5555555555555555ull;
    v = (v | (v >> 1)) & 0x3333333333333333ull;
    v = (v | (v >> 2)) & 0x0f0f0f0f0f0f0f0full;
    v = (v | (v >> 4)) & 0x00ff00ff00ff00ffull;
    v = (v | (v >> 8)) & 0x0000ffff0000ffffull;
    v = (v | (v >> 16)) & 0x00000000ffffffffull;
    return (uint32_t)v;
}

// Unit vector of the centre of nested pixel `pix` at nside = 2^level, before
// the user rotation.  The 12 base faces sit in three rows of four; inside a
// face the pixel's (px, py) come from the Z-order index.  The ring counted from
// the north pole is (row + 2) nside - px - py - 1; rings above nside and below
// 3 nside are polar-cap rings with 4*ring pixels, the others hold 4 nside.
__device__ inline void healpix_nest_dir(int level, uint32_t pix, double v[3]) {
    const int ns = 1 << level;
    const uint32_t face = pix >> (2 * level);
    const uint32_t in_face = pix & ((1u << (2 * level)) - 1u);
    const int px = (int)gather_even_bits(in_face);
    const int py = (int)gather_even_bits((uint64_t)in_face >> 1);
    const int row = (int)(face >> 2);
    const int col = (int)(face & 3u);
    const int ring = (row + 2) * ns - px - py - 1;
    double z, sin_theta;
    int ring_q;       // pixels in the ring / 4
    int half_shift;   // 1 if the ring's first pixel centre is at phi = 0
    const double inv3n2 = 1.0 / (3.0 * (double)ns * (double)ns);
    if (ring < ns) {
        ring_q = ring;
        const double t = (double)ring * (double)ring * inv3n2;  // 1 - z
        z = 1.0 - t;
        sin_theta = sqrt(t * (2.0 - t));
        half_shift = 0;
    } else if (ring > 3 * ns) {
        ring_q = 4 * ns - ring;
        const double t = (double)ring_q * (double)ring_q * inv3n2;  // 1 + z
        z = t - 1.0;
        sin_theta = sqrt(t * (2.0 - t));
        half_shift = 0;
    } else {
        ring_q = ns;
        z = (double)(2 * ns - ring) * (2.0 / (3.0 * (double)ns));
        sin_theta = sqrt((1.0 - z) * (1.0 + z));
        half_shift = (ring - ns) & 1;
    }
    // face column in units of half the in-ring spacing: odd for the polar rows
    const int face_col = 2 * col + ((row == 1) ? 0 : 1);
    int jp = (face_col * ring_q + px - py + 1 + half_shift) >> 1;
    if (jp > 4 * ring_q) jp -= 4 * ring_q;
    if (jp < 1) jp += 4 * ring_q;
    const double phi = ((double)jp - 0.5 * (double)(1 + half_shift)) * (M_PI * 0.5 / (double)ring_q);
    double s, c;
    sincos(phi, &s, &c);
    v[0] = sin_theta * c;
    v[1] = sin_theta * s;
    v[2] = z;
}

// ---------------------------------------------------------------------------
// Per-ray geometry and the march
// ---------------------------------------------------------------------------

struct Ray {
    double xs[3];     // source position
    double n[3];      // unit direction (rotated)
    double inv[3];    // 1/n (unused where n == 0)
    double r_a;       // start radius: 0 at level0, r_max(l-1) otherwise
    double r_end;     // r_split if the ray can split before leaving, else d_exit
    bool can_split;   // r_max(l) < d_exit (a tie exits)
    bool starts_outside;  // r_a >= d_exit: created outside the domain, no segment
    uint32_t dc[3];   // change of the linear cell index for one step along axis a (in direction n)
};

__device__ inline void ray_setup(const Geo& g, const double* __restrict__ src_pos, uint32_t src,
                                 int level, uint32_t pix, Ray& r) {
    double v[3];
    healpix_nest_dir(level, pix, v);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        r.xs[a] = src_pos[3 * src + a];
        r.n[a] = g.rot[3 * a + 0] * v[0] + g.rot[3 * a + 1] * v[1] + g.rot[3 * a + 2] * v[2];
        r.inv[a] = 1.0 / r.n[a];
    }
    const uint32_t stride[3] = {1u, (uint32_t)g.nx, (uint32_t)g.nx * (uint32_t)g.ny};
#pragma unroll
    for (int a = 0; a < 3; ++a) r.dc[a] = r.n[a] > 0.0 ? stride[a] : 0u - stride[a];
    const double hi[3] = {(double)g.nx, (double)g.ny, (double)g.nz};
    double d_exit = INFINITY;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        double t = INFINITY;
        if (r.n[a] > 0.0) t = (hi[a] - r.xs[a]) * r.inv[a];
        else if (r.n[a] < 0.0) t = (0.0 - r.xs[a]) * r.inv[a];
        d_exit = fmin(d_exit, t);
    }
    r.r_a = (level == g.level0) ? 0.0 : g.rmax[level - 1];
    const double r_split = (level < g.level_max) ? g.rmax[level] : INFINITY;
    r.can_split = r_split < d_exit;
    r.r_end = r.can_split ? r_split : d_exit;
    r.starts_outside = !(r.r_a < d_exit);
}

__device__ __forceinline__ bool source_inside(const Geo& g, const double* xs) {
    return xs[0] >= 0.0 && xs[0] < (double)g.nx && xs[1] >= 0.0 && xs[1] < (double)g.ny &&
           xs[2] >= 0.0 && xs[2] < (double)g.nz;
}

// Amanatides-Woo traversal of one ray from r_a to r_end, one segment per call,
// for loops that keep the whole wavefront converged between segments (the
// sweeps flush their deposit staging in converged code after every step).
// tau[] accumulates the optical depth of each bin from the source; the ray ends
// with kTerm as soon as tau_b > tau_term in every bin, else with kSplit / kExit
// on reaching r_end.  *stuck is set if the traversal failed to advance
// (non-finite input); the step count is bounded by the grid size, so every lane
// terminates.  The (n_H, x_n)
// pair of the next cell is loaded as soon as the ray steps into it, so the
// gather's latency overlaps the current segment's deposit.
struct MarchState {
    int cell[3];
    double tnext[3];
    double rr;
    uint32_t c;       // linear index of the current cell
    float2 q;         // (n_H, x_n) of the current cell
    float fg;         // the gas's share of the ionizing opacity in the current cell (if gathered)
    int it, max_steps;
    bool alive;
    int end;
};

// v_min_f64 / v_max_f64 without the NaN-quieting the compiler puts around
// fmin / fmax: face parameters are finite or +-infinity, never NaN.
__device__ __forceinline__ double min_f64(double x, double y) {
    double r;
    __asm__("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(x), "v"(y));
    return r;
}
__device__ __forceinline__ double max_f64(double x, double y) {
    double r;
    __asm__("v_max_f64 %0, %1, %2" : "=v"(r) : "v"(x), "v"(y));
    return r;
}

// Largest optical-depth increment one segment adds to a ray's running tau.  The
// transmission e^{-tau} is 0 in FP64 well before that, so no output changes,
// while the running sums keep their earlier terms: the adjoint recovers a
// segment's entry depth by subtracting its increment from the exit depth, which
// a single increment of ~1e36 would otherwise reduce to zero.  Above any
// termination depth art_create accepts.
constexpr double kTauStep = 1.0e6;

__device__ __forceinline__ uint32_t cell_index(const Geo& g, const int (&cell)[3]) {
    return ((uint32_t)cell[2] * (uint32_t)g.ny + (uint32_t)cell[1]) * (uint32_t)g.nx + (uint32_t)cell[0];
}

__device__ inline void march_begin(const Geo& g, const float2* __restrict__ q, const Ray& r, MarchState& m,
                                   const float* __restrict__ fg = nullptr) {
    const int dims[3] = {g.nx, g.ny, g.nz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double p = r.xs[a] + r.r_a * r.n[a];
        int c = (int)floor(p);
        c = c < 0 ? 0 : (c > dims[a] - 1 ? dims[a] - 1 : c);
        m.cell[a] = c;
        if (r.n[a] > 0.0) m.tnext[a] = ((double)(c + 1) - r.xs[a]) * r.inv[a];
        else if (r.n[a] < 0.0) m.tnext[a] = ((double)c - r.xs[a]) * r.inv[a];
        else m.tnext[a] = INFINITY;
    }
    m.rr = r.r_a;
    m.c = cell_index(g, m.cell);
    m.q = q[m.c];
    if (fg) m.fg = fg[m.c];
    m.it = 0;
    m.max_steps = g.nx + g.ny + g.nz + 8;
    m.alive = true;
    m.end = kExit;
}

// Advance one step, branch-free: every lane computes the candidate step and
// commits it only if it is alive, so the wavefront never splits around the
// march state.  Returns true if the lane produced a segment of positive length
// (then c, ijk, dr, dtau[], tau_in[] describe it and tau[] already includes
// it).  Clears m.alive and sets m.end when the ray is finished.
template <int NB>
__device__ __forceinline__ bool march_step(const Geo& g, const float2* __restrict__ q, const Ray& r,
                                           MarchState& m, double (&tau)[NB], bool* stuck, uint32_t& c,
                                           int (&ijk)[3], double& dr, double (&dtau)[NB], double (&tin)[NB],
                                           const float* __restrict__ fg = nullptr) {
    const int dims[3] = {g.nx, g.ny, g.nz};
    const bool alive = m.alive;
    const bool budget = m.it < m.max_steps;
    m.it += 1;
    const double rb0 = min_f64(min_f64(m.tnext[0], m.tnext[1]), m.tnext[2]);
    const bool ends = !(rb0 < r.r_end);
    const double rb = ends ? r.r_end : rb0;
    dr = rb - m.rr;
    const bool seg = alive & budget & (dr > 0.0);
    c = m.c;
#pragma unroll
    for (int a = 0; a < 3; ++a) ijk[a] = m.cell[a];
    const double dnH = (double)m.q.x;
    double kap[NB];
    kap[0] = dnH * ((double)m.q.y * g.s_H + g.s_d);
    if (NB > 1) kap[NB - 1] = dnH * g.s_d;
    bool thick = seg;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        dtau[b] = kap[b] * dr;
        tin[b] = tau[b];
        const double t1 = tau[b] + min_f64(dtau[b], kTauStep);
        tau[b] = seg ? t1 : tau[b];
        thick = thick & (t1 > g.tau_term);
    }
    m.rr = seg ? rb : m.rr;
    // step every axis whose face is at rb (ties step together)
    const bool go = alive & budget & !ends & !thick;
    bool moved = false, out = false;
    int nc[3];
    double nt[3];
    bool st[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        st[a] = m.tnext[a] == rb;
        const bool up = r.n[a] > 0.0;
        nc[a] = m.cell[a] + (up ? 1 : -1);
        const double face = (double)(up ? nc[a] + 1 : nc[a]);
        nt[a] = (face - r.xs[a]) * r.inv[a];
        moved = moved | st[a];
        // rounding guard at the boundary (the unsigned compare also catches nc < 0)
        out = out | (st[a] & ((uint32_t)nc[a] >= (uint32_t)dims[a]));
    }
    const bool adv = go & moved & !out;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const bool s2 = adv & st[a];
        m.cell[a] = s2 ? nc[a] : m.cell[a];
        m.tnext[a] = s2 ? nt[a] : m.tnext[a];
    }
    const bool bad = alive & (!budget | (go & !moved));
    *stuck = *stuck | bad;
    const bool finish = alive & !adv;
    const int end_new = thick ? kTerm : ((ends && r.can_split) ? kSplit : kExit);
    m.end = finish ? end_new : m.end;
    m.alive = alive & adv;
    uint32_t c2 = m.c;
#pragma unroll
    for (int a = 0; a < 3; ++a) c2 += (adv & st[a]) ? r.dc[a] : 0u;
    m.c = c2;
    if (adv) {  // prefetch for the next step
        m.q = q[c2];
        if (fg) m.fg = fg[c2];
    }
    return seg;
}

// The same segments walked backwards, from the last one to the first.  The
// entry face of a cell on an axis is the exit face the forward walk computed in
// the neighbouring cell, by the same expression ((face - x_s) / n_a), so the
// segment ends, ties (axes stepping together) and zero-length skips are those
// of march_step, in reverse order.  Starts in the cell of the ray's last segment,
// whose end is r_hi; ends at the ray's start r_a.  Optical depth is not tracked
// here (the caller has the forward's end value).
struct BackState {
    int cell[3];
    uint32_t start_c; // linear index of the forward walk's first cell (where the backward walk stops)
    double tprev[3];  // entry-face parameter of the current cell per axis
    double rhi;       // upper end of the current segment
    uint32_t c;
    float2 q;
    int it, max_steps;
    bool alive;
};

__device__ __forceinline__ double entry_face(const Ray& r, int a, int cell) {
    if (r.n[a] > 0.0) return ((double)cell - r.xs[a]) * r.inv[a];
    if (r.n[a] < 0.0) return ((double)(cell + 1) - r.xs[a]) * r.inv[a];
    return -INFINITY;
}

__device__ inline void back_begin(const Geo& g, const float2* __restrict__ q, const Ray& r, uint32_t last_cell,
                                  double r_last, BackState& m) {
    const uint32_t nxy = (uint32_t)g.nx * (uint32_t)g.ny;
    m.cell[2] = (int)(last_cell / nxy);
    const uint32_t rem = last_cell - (uint32_t)m.cell[2] * nxy;
    m.cell[1] = (int)(rem / (uint32_t)g.nx);
    m.cell[0] = (int)(rem - (uint32_t)m.cell[1] * (uint32_t)g.nx);
    const int dims[3] = {g.nx, g.ny, g.nz};
    int start[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        m.tprev[a] = entry_face(r, a, m.cell[a]);
        // the start cell exactly as march_begin finds it
        const double p = r.xs[a] + r.r_a * r.n[a];
        int c = (int)floor(p);
        start[a] = c < 0 ? 0 : (c > dims[a] - 1 ? dims[a] - 1 : c);
    }
    m.start_c = cell_index(g, start);
    m.rhi = r_last;
    m.c = last_cell;
    m.q = q[last_cell];
    m.it = 0;
    m.max_steps = g.nx + g.ny + g.nz + 8;
    m.alive = true;
}

// One segment backwards, branch-free like march_step.  Returns true if the lane
// produced a segment of positive length (c, ijk, dr, dtau describe it).
template <int NB>
__device__ __forceinline__ bool back_step(const Geo& g, const float2* __restrict__ q, const Ray& r, BackState& m,
                                          bool* stuck, uint32_t& c, int (&ijk)[3], double& dr, double (&dtau)[NB]) {
    const int dims[3] = {g.nx, g.ny, g.nz};
    const bool alive = m.alive;
    const bool budget = m.it < m.max_steps;
    m.it += 1;
    const double lo0 = max_f64(max_f64(m.tprev[0], m.tprev[1]), m.tprev[2]);
    // the ray's first segment: the forward's start cell (whose entry face can lie a
    // rounding error beyond r_a), or an entry face at or before r_a
    const bool first = (m.c == m.start_c) | !(lo0 > r.r_a);
    const double rlo = first ? r.r_a : lo0;
    dr = m.rhi - rlo;
    const bool seg = alive & budget & (dr > 0.0);
    c = m.c;
#pragma unroll
    for (int a = 0; a < 3; ++a) ijk[a] = m.cell[a];
    const double dnH = (double)m.q.x;
    double kap[NB];
    kap[0] = dnH * ((double)m.q.y * g.s_H + g.s_d);
    if (NB > 1) kap[NB - 1] = dnH * g.s_d;
#pragma unroll
    for (int b = 0; b < NB; ++b) dtau[b] = kap[b] * dr;
    const bool go = alive & budget & !first;
    bool moved = false, out = false;
    int nc[3];
    bool st[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        st[a] = m.tprev[a] == lo0;
        nc[a] = m.cell[a] - (r.n[a] > 0.0 ? 1 : -1);
        moved = moved | st[a];
        out = out | (st[a] & ((uint32_t)nc[a] >= (uint32_t)dims[a]));
    }
    const bool adv = go & moved & !out;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const bool s2 = adv & st[a];
        m.cell[a] = s2 ? nc[a] : m.cell[a];
        // entry_face() without its branches: an axis with n_a = 0 never steps
        // (its entry parameter stays -inf, below the others), so the value
        // computed for it here is never selected
        const double ef = ((double)(r.n[a] > 0.0 ? nc[a] : nc[a] + 1) - r.xs[a]) * r.inv[a];
        m.tprev[a] = s2 ? ef : m.tprev[a];
    }
    m.rhi = adv ? lo0 : m.rhi;
    *stuck = *stuck | (alive & (!budget | (go & (!moved | out))));
    m.alive = alive & adv;
    uint32_t c2 = m.c;
#pragma unroll
    for (int a = 0; a < 3; ++a) c2 -= (adv & st[a]) ? r.dc[a] : 0u;
    m.c = c2;
    if (adv) m.q = q[c2];
    return seg;
}

// (1 - e^{-x})/x and 1 - e^{-x} in FP32, accurate for small x (series below
// 0.1, where 1 - e^{-x} would cancel), branch-free.
__device__ __forceinline__ void absorb_factors(float x, float& phi, float& one_minus_e) {
#pragma clang fp contract(fast)
    const float ser = 1.0f - x * (0.5f - x * (1.0f / 6.0f - x * (1.0f / 24.0f - x * (1.0f / 120.0f))));
    const float ome = 1.0f - __expf(-x);
    const bool small = x < 0.1f;
    phi = small ? ser : ome * __builtin_amdgcn_rcpf(x);
    one_minus_e = small ? x * ser : ome;
}

// 1/d for normal d: the hardware estimate refined by two Newton steps (about
// 1 ulp), cheaper than a correctly rounded division.
__device__ __forceinline__ double rcp_f64(double d) {
    double r = __builtin_amdgcn_rcp(d);
    double t = fma(-d, r, 1.0);
    r = fma(r, t, r);
    t = fma(-d, r, 1.0);
    return fma(r, t, r);
}

// a * b + c as one three-operand v_fma_f64: with a constant c held in a
// register, the compiler's two-operand form would copy c first at every use.
__device__ __forceinline__ double fma3(double a, double b, double c) {
    double r;
    __asm__("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// e = e^{-x}, om = 1 - e^{-x} and einv = e^{+x} in FP64 for x >= 0, from one Cody and
// Waite reduction: k = rint(x / ln 2), y = k ln 2 - x in [-ln2/2, ln2/2] (ln 2 in two
// parts), e^{-x} = 2^{-k} e^{y} and e^{x} = 2^{k} e^{-y}.  e^{y} - 1 and e^{-y} - 1 share
// the even and odd parts of the Taylor series of e^{y} - 1 to degree 11 (truncation
// below 1e-14 relative): E(z) = z/2! + z^2/4! + ... + z^5/10!, O(z) = 1 + z/3! + ... +
// z^5/11!, z = y^2, e^{+-y} - 1 = E +- y O.  om = -(e^{y} - 1) when k = 0 (no
// cancellation), else 1 - e >= 0.29.  x is capped at 800; einv overflows to +inf
// beyond x ~ 709 (callers use it only where e is normal).
__device__ __forceinline__ void exp_neg_pos(double x, double& e, double& om, double& einv) {
    x = min_f64(x, 800.0);
    const double kd = rint(x * 1.4426950408889634);
    double y = fma(kd, 0x1.62e42feep-1, -x);
    y = fma(kd, 0x1.a39ef35793c76p-33, y);
    const double z = y * y;
    double ev = 1.0 / 3628800.0;  // 1/10!
    ev = fma3(ev, z, 1.0 / 40320.0);
    ev = fma3(ev, z, 1.0 / 720.0);
    ev = fma3(ev, z, 1.0 / 24.0);
    ev = fma(ev, z, 0.5);
    ev = ev * z;
    double od = 1.0 / 39916800.0;  // 1/11!
    od = fma3(od, z, 1.0 / 362880.0);
    od = fma3(od, z, 1.0 / 5040.0);
    od = fma3(od, z, 1.0 / 120.0);
    od = fma3(od, z, 1.0 / 6.0);
    od = fma(od, z, 1.0);
    const double yo = y * od;
    const double pp = ev + yo;  // e^{y} - 1
    const double pm = ev - yo;  // e^{-y} - 1
    const int k = (int)kd;
    e = ldexp(1.0 + pp, -k);
    einv = ldexp(1.0 + pm, k);
    om = kd == 0.0 ? -pp : 1.0 - e;
}

// FP64 versions for the adjoint: phi(x) = (1 - e^{-x})/x and
// phi'(x) = (x e^{-x} - (1 - e^{-x}))/x^2, given e = e^{-x} and om = 1 - e^{-x},
// with one reciprocal of x; series below 1e-3 (where x may be 0).
__device__ __forceinline__ void absorb_phi_dphi(double x, double e, double om, double& phi, double& dphi) {
    const bool small = x < 1e-3;
    const double r = rcp_f64(small ? 1.0 : x);
    phi = small ? 1.0 - x * (0.5 - x * (1.0 / 6.0 - x * (1.0 / 24.0))) : om * r;
    dphi = small ? -0.5 + x * (1.0 / 3.0 - x * (0.125 - x * (1.0 / 30.0))) : (x * e - om) * r * r;
}

// ---------------------------------------------------------------------------
// Wave-level helpers (wave64)
// ---------------------------------------------------------------------------

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

}  // namespace art
