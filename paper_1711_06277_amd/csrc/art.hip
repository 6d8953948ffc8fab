// art.hip -- MI355X (gfx950) implementation of the ART sweep behind the C ABI
// declared in include/art.h.
//
// Design (one GPU, one process):
//   * All sources of a call share one ray pool.  Rays live in per-HEALPix-level
//     segments of the pool, level l0 first, seeded by source and nested pixel;
//     after level l is swept, an order-preserving scan writes the children of its
//     splitting rays behind it in parent order, so every level stays sorted by
//     (source, direction) and the rays in flight cover a small part of the grid.
//     The pool holds the whole ray tree of a source wave (and doubles as the
//     adjoint's tape).  Sources are admitted in waves sized so that the tree of a
//     wave fits the pool.
//   * One persistent-style launch per level: a grid of resident workgroups whose
//     wavefronts claim 64-ray chunks from the level's shared multi-source queue
//     with one atomic per chunk, one ray per lane.  Rays of one level have the
//     same radial shell [r_max(l-1), r_max(l)], so the lanes of a wavefront do
//     similar amounts of work.
//   * Geometry, tau and all tree decisions in FP64; the per-segment deposit
//     arithmetic in FP32.  Deposits are merged per wavefront in an LDS cache of
//     64-bit fixed-point partial sums (LDS integer atomics are fast) and flushed
//     with coalesced global atomics: 64-bit integers in the deterministic mode
//     (integer sums do not depend on the order, so results are bitwise
//     reproducible), FP32 otherwise.
//   * The destroy counter of Sec. 2.2 (a ray ended at level l adds
//     4^(l_max - l)) is kept as a device-side completeness check of the tree.
//   * No allocation, host synchronisation or memset node inside art_trace /
//     art_trace_adjoint: they can be captured into a HIP graph.
#include <hip/hip_runtime.h>

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "art_device.h"

using namespace art;

namespace {

// --------------------------------------------------------------------------
// Device state
// --------------------------------------------------------------------------

// Counters of the current source wave, reset by the seed kernel.
struct WaveCounters {
    uint32_t head[ART_MAX_LEVELS + 1];      // forward chunk claims per level
    uint32_t tail[ART_MAX_LEVELS + 1];      // rays per level (set by the child scan of the level above)
    uint32_t adj_head[ART_MAX_LEVELS + 1];  // adjoint chunk claims per level
    uint64_t off[ART_MAX_LEVELS + 1];       // pool offset of each level
};

// Counters of a whole call.
struct CallCounters {
    unsigned long long destroy;
    unsigned long long segments;
    unsigned long long rays_wave_max;
    uint32_t status;
    uint32_t waves;               // source waves that traced at least one source
    double scale, inv_scale;      // forward fixed point: ~2^50 / L_total
    double gscale[2], inv_gscale[2];  // adjoint fixed point: dL/dn_H, dL/dx_n
};

struct Counters {
    WaveCounters w;
    CallCounters c;
};

// Parents per tile of the child scan: whole claims of kWave rays.
constexpr int kSplitTile = 4096;
static_assert(kSplitTile % kWave == 0, "a claim lies in one tile");

// The ray pool, structure of arrays.
struct Pool {
    uint32_t* src;    // source index
    uint32_t* pix;    // nested pixel at the ray's level
    double* tau;      // [cap][2]: optical depth from the source at the ray's start
    uint32_t* child;  // pool index of the first of the four children (or kNoChild)
    double* G;        // [cap][2]: adjoint, loss contributed downstream of the start; the same
                      // memory as tau, which no adjoint reads and the next forward reseeds
    double* tend;     // [cap][2]: optical depth where a splitting ray split; -1 if it did not
    // adjoint tape (NULL without adjoint support): the cell of each ray's last
    // segment (kNoChild if it has none), that segment's upper end, and the
    // optical depth at the ray's end
    uint32_t* last;
    double* rlast;
    double* taulast;  // [cap][2]
    uint32_t* tsum;   // splitting rays per tile of kSplitTile parents (counted by the sweep), then
                      // their exclusive prefix; all zero between levels
    uint64_t cap;
};

// Per-source statistics, [max_src][ART_MAX_LEVELS] / [max_src][2] / [max_src].
struct SrcStats {
    uint32_t *created, *split, *exited, *term;
    double *escaped, *residual;
    unsigned long long* segments;
};

// Clears every per-source counter of a call in one launch.
__global__ void k_zero_stats(SrcStats st, uint64_t ms) {
    const uint64_t n_lev = ms * ART_MAX_LEVELS;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n_lev;
         i += (uint64_t)gridDim.x * blockDim.x) {
        st.created[i] = 0u;
        st.split[i] = 0u;
        st.exited[i] = 0u;
        st.term[i] = 0u;
        if (i < 2 * ms) {
            st.escaped[i] = 0.0;
            st.residual[i] = 0.0;
        }
        if (i < ms) st.segments[i] = 0ull;
    }
}

struct SweepArgs {
    Geo g;
    const float2* q;   // (n_H, x_n) per cell, packed once per call
    const float* fg;   // gas share of the ionizing opacity per cell
    const float* nH;
    const float* xn;
    const double* src_pos;
    const float* src_lum;
    Pool pool;
    Counters* ct;
    SrcStats st;
    // deposit accumulators, one cell's values contiguous (AoS, stride 4 or 8):
    // J0, Fx, Fy, Fz[, J1]; FP32 (atomic mode) or 64-bit fixed point
    float* acc;
    unsigned long long* det;
    uint32_t N;
    uint32_t n_src;
};

struct AdjArgs {
    Geo g;
    const float2* q;   // (n_H, x_n) per cell
    const float4* wv;  // (w, v_x, v_y, v_z) per cell: the weights of rate and force in L
    const double* src_pos;
    const float* src_lum;
    Pool pool;
    Counters* ct;
    double* gk;                // [N][2] (dL/dn_H, dL/dx_n) per cell, FP64
    unsigned long long* gdet;  // [N][2] the same in fixed point
    uint32_t N;
    uint32_t n_src;
};

// Round x * scale to the nearest 64-bit integer (ties to even), for |x * scale| <
// 2^51: adding 1.5 * 2^52 in one FP64 rounding puts the integer in the low bits of
// the significand (the sum stays in [2^52, 2^53), where the spacing is 1), so the
// integer is the sum's bit pattern minus that of 1.5 * 2^52.
__device__ __forceinline__ long long fixed_point(float x, double scale) {
    return __double_as_longlong(fma((double)x, scale, 0x1.8p52)) - 0x4338000000000000ll;
}


// --------------------------------------------------------------------------
// Small kernels
// --------------------------------------------------------------------------

__global__ void k_fill_u32(uint32_t* p, uint64_t n, uint32_t v) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_u64(unsigned long long* p, uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

__global__ void k_fill_f32(float* p, uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

__global__ void k_fill_f64(double* p, uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0.0;
}

// Interleave (n_H, x_n) so that the sweep gathers one 8-byte word per segment.
// transparent (optional): cells of sink control volumes, whose gas the radiation
// ignores (no gas as far as the sweep is concerned).
// The fields are also checked here (the pass reads every cell anyway): a cell with
// n_H < 0 or not finite, or x_n outside [0, 1], sets kStBadField.
// fg[c] = x_n s_H / (x_n s_H + s_d): the gas's share of the ionizing bin's opacity,
// which turns a segment's absorbed ionizing luminosity into its photoionizations
// (Eq. e:photrate2); 0 where nothing absorbs.
__global__ void k_pack(uint64_t N, const float* nH, const float* xn, const uint8_t* transparent, float2* q,
                       float* fg, double s_H, double s_d, Counters* ct) {
    bool bad = false;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < N;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const float n = nH[i], x = xn[i];
        bad = bad || !(n >= 0.0f && n <= 3.4e38f) || !(x >= 0.0f && x <= 1.0f);
        const bool sink = transparent && transparent[i];
        q[i] = make_float2(sink ? 0.0f : n, x);
        const double gas = (double)x * s_H, chi = gas + s_d;
        fg[i] = (sink || !(chi > 0.0)) ? 0.0f : (float)(gas / chi);
    }
    if (__ballot(bad) && lane_id() == 0) atomicOr(&ct->c.status, (uint32_t)kStBadField);
}

// The adjoint's per-cell weights in one 16-byte gather: (w, v_x, v_y, v_z).
__global__ void k_pack_wv(uint64_t N, const float* w, const float* v, float4* wv) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < N;
         i += (uint64_t)gridDim.x * blockDim.x)
        wv[i] = make_float4(w[i], v[i], v[N + i], v[2 * N + i]);
}

// Reset the call counters and set the fixed-point scale of the deposits, a power
// of two 2^k, as fine as two bounds allow:
//   * one quantised value (a lane's deposit after the quad pre-combine) must
//     stay below 2^50 so that fixed_point() converts it exactly.  A lane's value
//     is at most sqrt(3) L_nom(l) summed over bins (a segment is at most a cell
//     diagonal long, phi <= 1, the packet never grows), L_nom(l) <= L_s / (12 4^l0),
//     and the combine adds at most the four lanes of a quad:
//     D = 4 sqrt(3) max_s(sum_b L_s,b) / (12 4^l0);
//   * a cell's sum must stay below 2^62: from one source, the rays of one level
//     carry at most L_s in all and cross a cell once each (at most sqrt(3)), and a
//     cell (radial extent sqrt(3)) meets at most n_shell levels' shells:
//     S = n_shell sqrt(3) L_total.
// Both get a margin of 2^-10 for the FP32 rounding of the values.
__global__ void k_begin_call(Counters* ct, const float* src_lum, int n_src, int n_bins, int level0, int n_shell) {
    __shared__ double part[256], pmax[256];
    double s = 0.0, mx = 0.0;
    for (int i = threadIdx.x; i < n_src; i += blockDim.x) {
        double ls = 0.0;
        for (int b = 0; b < n_bins; ++b) ls += fabs((double)src_lum[(uint64_t)i * n_bins + b]);
        s += ls;
        mx = fmax(mx, ls);
    }
    part[threadIdx.x] = s;
    pmax[threadIdx.x] = mx;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            part[threadIdx.x] += part[threadIdx.x + o];
            pmax[threadIdx.x] = fmax(pmax[threadIdx.x], pmax[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double L = part[0] > 0.0 ? part[0] : 1.0;
        const double Lmax = pmax[0] > 0.0 ? pmax[0] : 1.0;
        ct->c.destroy = 0ull;
        ct->c.segments = 0ull;
        ct->c.rays_wave_max = 0ull;
        ct->c.status = 0u;
        ct->c.waves = 0u;
        const double margin = 1.0 + 0x1p-10;
        const double D = 4.0 * 1.7320508075688772 * Lmax / (12.0 * ldexp(1.0, 2 * level0)) * margin;
        const double S = (double)n_shell * 1.7320508075688772 * L * margin;
        // x < 2^(ilogb(x) + 1): D 2^(50 - ilogb(D) - 1) < 2^50, S 2^(62 - ilogb(S) - 1) < 2^62
        int k = min(50 - ilogb(D) - 1, 62 - ilogb(S) - 1);
        k = k > 900 ? 900 : (k < -900 ? -900 : k);
        ct->c.scale = ldexp(1.0, k);
        ct->c.inv_scale = ldexp(1.0, -k);
    }
}

// Fixed-point scale of the adjoint.  Per cell, |dL/dkappa_b| <= 4 W L_total with
// W = max w + sqrt(3) max |v| (every downstream contribution of a ray is at
// most W times its packet, and sum over rays of packet x dr is at most the
// vacuum J <= sqrt(3) L_total); dL/dn_H and dL/dx_n add the chain-rule factors
// (x_n s_H + s_d) <= s_H + s_d and n_H s_H <= max(n_H) s_H.  scratch[0] = W,
// scratch[1] = max n_H (float bit patterns, non-negative, so unsigned max works).
__global__ void k_adj_scale(const float* w, const float* v, const float* nH, uint64_t N, float* scratch) {
    __shared__ float pw[256], pn[256];
    float m = 0.0f, mn = 0.0f;
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < N;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const float vv = fabsf(v[i]) + fabsf(v[N + i]) + fabsf(v[2 * N + i]);
        m = fmaxf(m, fabsf(w[i]) + 1.7320508f * vv);
        mn = fmaxf(mn, fabsf(nH[i]));
    }
    pw[threadIdx.x] = m;
    pn[threadIdx.x] = mn;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            pw[threadIdx.x] = fmaxf(pw[threadIdx.x], pw[threadIdx.x + o]);
            pn[threadIdx.x] = fmaxf(pn[threadIdx.x], pn[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicMax((unsigned int*)&scratch[0], __float_as_uint(pw[0]));
        atomicMax((unsigned int*)&scratch[1], __float_as_uint(pn[0]));
    }
}

__global__ void k_adj_scale_final(Counters* ct, const float* src_lum, int n_lum, const float* scratch,
                                  double s_H, double s_d) {
    if (threadIdx.x != 0) return;
    double L = 0.0;
    for (int i = 0; i < n_lum; ++i) L += fabs((double)src_lum[i]);
    if (!(L > 0.0)) L = 1.0;
    double W = (double)scratch[0];
    if (!(W > 0.0)) W = 1.0;
    // dL/dkappa_b of a segment is bounded without reference to n_H; dL/dn_H takes
    // it times (x_n s_H + s_d) or s_d, dL/dx_n times n_H s_H, so only the latter
    // bound carries the largest density
    const double chain[2] = {1.0 + s_H + s_d, 1.0 + s_H + s_d + s_H * (double)scratch[1]};
    for (int i = 0; i < 2; ++i) {
        const double bound = 8.0 * W * L * chain[i];
        ct->c.gscale[i] = ldexp(1.0, 58) / bound;
        ct->c.inv_gscale[i] = bound * ldexp(1.0, -58);
    }
}

// Seed a source wave: 12*4^l0 rays per source at level l0 (Sec. 2.1), source
// major and nested pixel minor, so that a wavefront holds 64 neighbouring
// directions of one source.  Resets the wave counters.
// With a wave table (planned on the device), wave w traces sources
// wtab[w] .. wtab[w + 1] - 1 and src0 / n_wave are ignored; past the last planned
// wave it seeds nothing, and every later launch of the wave finds no rays.
__global__ void k_seed(Pool pool, Counters* ct, int level0, int src0, int n_wave, const int* wtab, int w,
                       int want_child) {
    const uint32_t per_src = 12u << (2 * level0);
    if (wtab) {
        src0 = wtab[w];
        n_wave = wtab[w + 1] - src0;
    }
    const uint64_t n = (uint64_t)per_src * (uint64_t)n_wave;
    if (blockIdx.x == 0 && threadIdx.x == 0 && n_wave > 0) atomicAdd(&ct->c.waves, 1u);
    if (blockIdx.x == 0 && threadIdx.x <= ART_MAX_LEVELS) {
        const int l = threadIdx.x;
        ct->w.head[l] = 0u;
        ct->w.adj_head[l] = 0u;
        ct->w.tail[l] = (l == level0) ? (uint32_t)n : 0u;
        ct->w.off[l] = 0ull;
    }
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        pool.src[i] = (uint32_t)src0 + (uint32_t)(i / per_src);
        pool.pix[i] = (uint32_t)(i % per_src);
        pool.tau[2 * i] = 0.0;
        pool.tau[2 * i + 1] = 0.0;
        if (want_child) pool.child[i] = kNoChild;
    }
    // the sweeps count splitting rays per tile into zeroed counters, and every
    // scatter clears the tiles it used
    const uint64_t n_tiles = (pool.cap + kSplitTile - 1) / kSplitTile + 1;
    for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < n_tiles;
         t += (uint64_t)gridDim.x * blockDim.x)
        pool.tsum[t] = 0u;
}

// ---------------------------------------------------------------------------
// Source waves planned on the device
// ---------------------------------------------------------------------------

// Pixels of the coarse levels are tested one by one; deeper levels through
// their level-kBoundLevel ancestors.
constexpr int kBoundLevel = 6;
constexpr uint32_t kDirTable = 12u * ((1u << (2 * (kBoundLevel + 1))) - 1u) / 3u;  // levels 0..kBoundLevel

__host__ __device__ constexpr uint32_t dir_offset(int level) { return 12u * ((1u << (2 * level)) - 1u) / 3u; }

// Unrotated HEALPix pixel centres of levels 0..kBoundLevel, level by level.
__global__ void k_dir_table(double* dirs) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < kDirTable; i += gridDim.x * blockDim.x) {
        int l = 0;
        while (l < kBoundLevel && i >= dir_offset(l + 1)) ++l;
        double v[3];
        healpix_nest_dir(l, i - dir_offset(l), v);
        dirs[3 * i] = v[0];
        dirs[3 * i + 1] = v[1];
        dirs[3 * i + 2] = v[2];
    }
}

// An upper bound on the rays one source creates (one workgroup per source).  A
// level-l ray exists only if its parent split, i.e. if the parent's direction
// at r_max(l-1) is strictly inside the box (Sec. 2.1; its ancestors must have
// split too, so counting all level-(l-1) directions is a bound).  Levels up to
// kBoundLevel are counted pixel by pixel; a deeper level's pixels are counted
// through their level-kBoundLevel ancestors, whose descendants' directions lie
// within twice the mean pixel spacing sqrt(4 pi / N_pix) of the ancestor's (the
// largest distance is about one spacing), so an ancestor counts all of them if
// its point at r_max(l-1) is within that angle times r_max(l-1) of the box.
// Capped by `loose`, the geometric bound the pool was sized with.
__global__ void __launch_bounds__(256) k_src_bound(Geo g, const double* __restrict__ src_pos, int n_src,
                                                   const double* __restrict__ dirs, int deepest,
                                                   unsigned long long loose, unsigned long long* bound) {
    __shared__ uint32_t part[256 / kWave];
    const int s = blockIdx.x;
    if (s >= n_src) return;
    const double xs[3] = {src_pos[3 * s], src_pos[3 * s + 1], src_pos[3 * s + 2]};
    const double hi[3] = {(double)g.nx, (double)g.ny, (double)g.nz};
    unsigned long long tot = 12ull << (2 * g.level0);
    for (int l = g.level0 + 1; l <= deepest; ++l) {
        const int L = l - 1, Lc = L < kBoundLevel ? L : kBoundLevel;
        const double R = g.rmax[L];
        const double spacing = sqrt(4.0 * M_PI / (double)(12u << (2 * Lc)));
        const double pad = (L > Lc ? 2.0 * spacing * R : 0.0) + 1e-6 * (R + 1.0);
        const uint32_t npix = 12u << (2 * Lc);
        const double* d = dirs + 3 * (uint64_t)dir_offset(Lc);
        uint32_t cnt = 0;
        for (uint32_t p = threadIdx.x; p < npix; p += blockDim.x) {
            bool in = true;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double u = g.rot[3 * a] * d[3 * p] + g.rot[3 * a + 1] * d[3 * p + 1] + g.rot[3 * a + 2] * d[3 * p + 2];
                const double x = xs[a] + R * u;
                in = in && x > -pad && x < hi[a] + pad;
            }
            cnt += in ? 1u : 0u;
        }
        cnt = wave_sum(cnt);
        if (lane_id() == 0) part[threadIdx.x / kWave] = cnt;
        __syncthreads();
        unsigned long long c = 0;
        for (int k = 0; k < (int)(blockDim.x / kWave); ++k) c += part[k];
        __syncthreads();
        const unsigned long long rays = 4ull * c << (2 * (L - Lc));
        tot += rays < (12ull << (2 * l)) ? rays : (12ull << (2 * l));
    }
    if (threadIdx.x == 0) bound[s] = tot < loose ? tot : loose;
}

// Consecutive sources into waves whose bounds add up to at most `cap` rays (a
// source whose bound alone exceeds it gets a wave of its own): wave w is
// sources wtab[w] .. wtab[w + 1] - 1; entries past the last wave repeat n_src.
// At most max_waves waves (the fixed-size plan's count, which this never exceeds
// because every bound is at most the one that plan assumed).
__global__ void k_plan_waves(const unsigned long long* bound, int n_src, unsigned long long cap, int max_waves,
                             int* wtab) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int w = 0, s = 0;
    while (s < n_src) {
        wtab[w++] = s;
        if (w == max_waves) {  // not reached (see above); the last wave would take the rest
            s = n_src;
            break;
        }
        unsigned long long acc = 0;
        while (s < n_src && (acc == 0 || acc + bound[s] <= cap)) acc += bound[s++];
    }
    for (int k = w; k <= max_waves; ++k) wtab[k] = n_src;
}

// --------------------------------------------------------------------------
// Per-wavefront LDS write-back cache of deposits
// --------------------------------------------------------------------------

// The 64 lanes of a wavefront trace neighbouring directions of one source, so
// their segments keep landing in the same few cells.  Global atomics cost one
// memory transaction per cache line touched (scattered single-lane atomics run
// ~15x slower than atomics on 64 consecutive words), so deposits go through
// two stages in LDS:
//   1. a direct-mapped cache of S cells (slot = the cell's position in an
//      8 x 8 x (S/64) tile) accumulated with LDS atomics;
//   2. cells evicted from it (or that lost a slot) are appended to a staging
//      list, which the whole wavefront flushes in converged code: lane l adds
//      value (l mod LPE) of staged cell (l / LPE), so the NV values of a cell,
//      contiguous in the AoS accumulator, share one memory transaction.
// Both LDS arrays hold one row per value (slot h of value q at q * S + h): the
// lanes of a wavefront address scattered slots, and with 8-byte values a
// slot-major layout (stride 32 bytes) maps slots 0, 8, 16, ... onto the same
// banks.  Every wavefront takes its part of the workgroup's dynamic LDS, so a
// 64-thread workgroup needs a quarter of what a 256-thread one does.
// Every step is executed in program order by the active lanes of one
// wavefront and LDS executes a wavefront's instructions in order, so no barrier
// is needed between lanes; compiler barriers keep the order of the LDS
// operations of lanes in different branches.
constexpr uint32_t kEmptyKey = 0xffffffffu;
#define ART_LDS __attribute__((address_space(3)))

// LDS atomic add at wavefront scope (a cache belongs to one wavefront).
template <class T>
__device__ __forceinline__ void lds_add(ART_LDS T* p, T x) {
    __hip_atomic_fetch_add(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
__device__ __forceinline__ void global_add(double* p, double x) { unsafeAtomicAdd(p, x); }
__device__ __forceinline__ void global_add(unsigned long long* p, unsigned long long x) { atomicAdd(p, x); }

// Compiler-only barrier: LDS operations of different lanes in different
// branches are not reordered across it.
__device__ __forceinline__ void lds_order() { __asm__ volatile("" ::: "memory"); }

// A register the compiler treats as written, with no instruction: for values read
// only on paths that assign them first.  Left undefined instead, such arrays are
// zero-filled on every loop iteration, one move per register.
template <class T> __device__ __forceinline__ T unset() {
    T x;
    __asm__ volatile("" : "=v"(x));
    return x;
}

template <int NV, class V_, int S_>
struct Deposit {
    using V = V_;  // double, or unsigned 64-bit fixed point (two's complement sums)
    static constexpr int S = S_;           // cache slots: 128 or 256
    static_assert(S_ == 128 || S_ == 256, "the slot map is an 8 x 8 x (S/64) tile");
    static_assert(S % kWave == 0, "init and drain walk the slots a wavefront at a time");
    static constexpr int W = NV;           // values per slot
    static constexpr int CAP = 128;        // staging capacity (>= 64 + flush threshold)
    static constexpr uint32_t kFlushAt = CAP - kWave;
    // Staging row stride: the flush reads rows f = 0..3 at one column each; a
    // stride of 144 words puts those rows 16 (FP32) or 32 (64-bit) banks apart.
    static constexpr int CAPP = CAP + 16;
    static constexpr int LPE = NV <= 2 ? 2 : (NV <= 4 ? 4 : 8);  // AoS stride of the accumulator = lanes per staged cell
    // LDS bytes per wavefront: values first (8-byte aligned), then the keys
    static constexpr size_t kBytes = sizeof(V) * (size_t)NV * (S + CAPP) + sizeof(uint32_t) * (S + CAP);
    ART_LDS uint32_t* keys;                // [S]
    ART_LDS V* vals;                       // [NV][S]: value q of slot h at q * S + h
    ART_LDS uint32_t* skey;                // [CAP]
    ART_LDS V* sval;                       // [NV][CAPP]
    uint32_t n_staged;                     // wave-uniform

    // Carve the wavefront's part out of the workgroup's dynamic LDS.
    __device__ static inline Deposit at(unsigned char* base) {
        ART_LDS unsigned char* b = (ART_LDS unsigned char*)base;
        ART_LDS V* v = (ART_LDS V*)b;
        ART_LDS V* sv = v + (size_t)NV * S;
        ART_LDS uint32_t* k = (ART_LDS uint32_t*)(sv + (size_t)NV * CAPP);
        return Deposit{k, v, k + S, sv, 0u};
    }

    // The cell's position in an 8 x 8 x (S/64) tile, with the tile's upper bits
    // folded into the lower ones (a bijection): the lanes of a wavefront cross a
    // patch of neighbouring cells, and without the fold cells that differ only in k
    // (or in the high bit of j) would share LDS banks.
    __device__ static inline uint32_t slot(const int (&ijk)[3]) {
        const uint32_t h = (uint32_t)((ijk[0] & 7) | ((ijk[1] & 7) << 3) | ((ijk[2] & (S / 64 - 1)) << 6));
        return h ^ ((h >> 4) & (uint32_t)(S / 16 - 1));
    }
    __device__ inline void init(int lane) {
        for (int s = lane; s < S; s += kWave) keys[s] = kEmptyKey;
        n_staged = 0u;
        lds_order();
    }

    // Active lanes only (any subset of the wavefront).  A lane whose cell hits
    // the slot's key adds into LDS.  Otherwise it tries to swap its cell into
    // the slot (LDS compare-and-swap: of several lanes one wins); the winner
    // hands back the slot's previous cell and values, to be staged for global
    // memory, and initialises the slot with its own values; lanes that lost to
    // a lane with the same cell add after that; any other lane hands back its
    // own deposit.  Returns true if (pk, pv) must be staged.
    __device__ inline bool deposit(uint32_t c, const int (&ijk)[3], const V (&v)[NV], uint32_t& pk, V (&pv)[NV]) {
        const uint32_t h = slot(ijk);
        ART_LDS V* sv = vals + h;
        const uint32_t key0 = keys[h];
        const bool hit = key0 == c;
        if (hit) {
#pragma unroll
            for (int q = 0; q < NV; ++q) lds_add(&sv[q * S], v[q]);
        }
        // Lanes that hit and lanes that evict run mutually exclusive branches,
        // so nothing orders them for the compiler: keep every add issued before
        // any eviction (LDS then executes them in issue order).
        lds_order();
        bool pend = false;
        uint32_t prev = key0;
        if (!hit) prev = atomicCAS((uint32_t*)&keys[h], key0, c);
        const bool won = !hit && prev == key0;
        if (won) {  // won the slot: evict the previous cell, initialise with ours
            pk = key0;
            pend = key0 != kEmptyKey;
#pragma unroll
            for (int q = 0; q < NV; ++q) pv[q] = sv[q * S];
#pragma unroll
            for (int q = 0; q < NV; ++q) sv[q * S] = v[q];
        }
        // lanes that lost the slot to a lane with the same cell add after the
        // winner has initialised it
        lds_order();
        const bool follower = !hit && !won && prev == c;
        if (follower) {
#pragma unroll
            for (int q = 0; q < NV; ++q) lds_add(&sv[q * S], v[q]);
        }
        if (!hit && !won && !follower) {
            pk = c;
#pragma unroll
            for (int q = 0; q < NV; ++q) pv[q] = v[q];
            pend = true;
        }
        lds_order();
        return pend;
    }

    // Converged: append the lanes' pending entries to the staging list.
    __device__ inline void stage(bool pend, uint32_t pk, const V (&pv)[NV]) {
        const unsigned long long mk = __ballot(pend);
        lds_order();
        if (pend) {
            const uint32_t e = n_staged + (uint32_t)__builtin_amdgcn_mbcnt_hi(
                                              (uint32_t)(mk >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mk, 0u));
            skey[e] = pk;
#pragma unroll
            for (int q = 0; q < NV; ++q) sval[q * CAPP + e] = pv[q];
        }
        n_staged += (uint32_t)__popcll(mk);
        lds_order();
    }

    // Converged: the whole wavefront writes the staged cells to the AoS
    // accumulator (stride LPE) when at least `threshold` are staged: lane l adds
    // value (l mod LPE) of staged cell (l / LPE).
    __device__ inline void flush(V* acc, int lane, uint32_t threshold) {
        const uint32_t n = n_staged;
        if (n < threshold || n == 0) return;
        const uint32_t per = kWave / LPE;
        const int f = lane % LPE;
        for (uint32_t b0 = 0; b0 < n; b0 += per) {
            const uint32_t e = b0 + (uint32_t)lane / LPE;
            if (e < n && f < NV) {
                global_add(acc + (uint64_t)skey[e] * LPE + f, sval[f * CAPP + e]);
            }
        }
        n_staged = 0u;
        lds_order();
    }

    // Converged: empty the cache into the accumulator.  Fewer than kFlushAt cells
    // may be staged on entry (each pass stages up to 64 more).
    __device__ inline void drain(V* acc, int lane) {
        for (int s0 = 0; s0 < S; s0 += kWave) {
            const int s = s0 + lane;
            const uint32_t k = keys[s];
            V old[NV];
#pragma unroll
            for (int q = 0; q < NV; ++q) old[q] = vals[q * S + s];
            stage(k != kEmptyKey, k, old);
            keys[s] = kEmptyKey;
            lds_order();
            flush(acc, lane, 1u);
        }
    }
};

// A slot holding a group of G cells, G g .. G g + G - 1, whose values are
// adjacent in the AoS accumulator (the forward sweep's fixed point uses G = 2:
// one 64-byte segment of two cells x four 8-byte values).  Memory-side atomics
// cost per request, and the lanes of one flush instruction on one segment make
// one request, so an evicted group reaches memory in one request; neighbouring
// cells along x also share a slot, which cuts the evictions themselves.  The
// staging list holds groups (one key, and the values in planes by value and
// cell, so consecutive groups are consecutive words); a flush instruction
// covers whole groups.
template <int NV, class V_, int G_>
struct GroupDeposit {
    using V = V_;
    static constexpr int G = G_;
    static_assert(G == 2 || G == 4, "groups of 2 or 4 cells");
    static constexpr int S = 64;           // slots: a 4 x 4 x 4 tile of (i / G, j, k), folded
    static_assert(S % kWave == 0, "init and drain walk the slots a wavefront at a time");
    static constexpr int W = G * NV;       // values per slot (cell G g first)
    static constexpr int CAP = G * kWave + 16;  // staged cells: a step adds at most G x 64, and
                                                // stages only after a flush left < kFlushAt
    static constexpr uint32_t kFlushAt = CAP - G * kWave;
    static constexpr int CAPG = CAP / G;                  // staged groups
    static constexpr int CAPH = CAPG + 4;                 // plane stride
    static constexpr int LPE = NV <= 2 ? 2 : (NV <= 4 ? 4 : 8);
    static_assert((kWave / LPE) % G == 0, "a flush instruction covers whole groups");
    static constexpr size_t kBytes = sizeof(V) * ((size_t)W * S + (size_t)W * CAPH) + sizeof(uint32_t) * (S + CAPG);
    ART_LDS uint32_t* keys;                // [S]: group index g, or kEmptyKey
    ART_LDS V* vals;                       // [W][S]: value q of cell G g + s in slot h at (s * NV + q) * S + h
    ART_LDS uint32_t* skey;                // [CAPG]: staged group keys
    ART_LDS V* sval;                       // [NV][G][CAPH]: value q of cell s of staged group p at (q * G + s) * CAPH + p
    uint32_t n_staged;                     // staged cells, wave-uniform, a multiple of G

    __device__ static inline GroupDeposit at(unsigned char* base) {
        ART_LDS unsigned char* b = (ART_LDS unsigned char*)base;
        ART_LDS V* v = (ART_LDS V*)b;
        ART_LDS V* sv = v + (size_t)W * S;
        ART_LDS uint32_t* k = (ART_LDS uint32_t*)(sv + (size_t)W * CAPH);
        return GroupDeposit{k, v, k + S, sv, 0u};
    }
    // k's bits folded into the i bits (a bijection): with 8-byte rows of 64
    // slots, slots 32 apart share LDS banks.
    __device__ static inline uint32_t slot(const int (&ijk)[3]) {
        const uint32_t h = (((uint32_t)ijk[0] / G) & 3u) | (((uint32_t)ijk[1] & 3u) << 2) | (((uint32_t)ijk[2] & 3u) << 4);
        return h ^ ((h >> 4) & 3u);
    }

    __device__ inline void init(int lane) {
        for (int s = lane; s < S; s += kWave) keys[s] = kEmptyKey;
        n_staged = 0u;
        lds_order();
    }

    // Active lanes only.  As Deposit::deposit, keyed by the group; a winner
    // starts its slot with its own values in its part and zeros elsewhere.
    // Returns true if the group (pk, pv) must be staged.
    __device__ inline bool deposit(uint32_t c, const int (&ijk)[3], const V (&v)[NV], uint32_t& pk, V (&pv)[W]) {
        const uint32_t g = c / (uint32_t)G;
        const uint32_t part = c % (uint32_t)G;
        const uint32_t own = part * (uint32_t)NV;
        const uint32_t h = slot(ijk);
        ART_LDS V* sv = vals + h;
        const uint32_t key0 = keys[h];
        const bool hit = key0 == g;
        if (hit) {
#pragma unroll
            for (int q = 0; q < NV; ++q) lds_add(&sv[(own + q) * S], v[q]);
        }
        lds_order();
        bool pend = false;
        uint32_t prev = key0;
        if (!hit) prev = atomicCAS((uint32_t*)&keys[h], key0, g);
        const bool won = !hit && prev == key0;
        if (won) {
            pk = key0;
            pend = key0 != kEmptyKey;
#pragma unroll
            for (int w = 0; w < W; ++w) pv[w] = sv[w * S];
            if constexpr (G == 2) {
                const uint32_t other = (uint32_t)NV - own;
#pragma unroll
                for (int q = 0; q < NV; ++q) {
                    sv[(own + q) * S] = v[q];
                    sv[(other + q) * S] = (V)0;
                }
            } else {
#pragma unroll
                for (int s = 0; s < G; ++s)
#pragma unroll
                    for (int q = 0; q < NV; ++q) sv[(s * NV + q) * S] = (uint32_t)s == part ? v[q] : (V)0;
            }
        }
        lds_order();
        const bool follower = !hit && !won && prev == g;
        if (follower) {
#pragma unroll
            for (int q = 0; q < NV; ++q) lds_add(&sv[(own + q) * S], v[q]);
        }
        if (!hit && !won && !follower) {
            pk = g;
#pragma unroll
            for (int s = 0; s < G; ++s)
#pragma unroll
                for (int q = 0; q < NV; ++q) pv[s * NV + q] = (uint32_t)s == part ? v[q] : (V)0;
            pend = true;
        }
        lds_order();
        return pend;
    }

    // Converged: append the pending groups (G entries each) to the staging list.
    __device__ inline void stage(bool pend, uint32_t pk, const V (&pv)[W]) {
        const unsigned long long mk = __ballot(pend);
        lds_order();
        if (pend) {
            const uint32_t p = n_staged / (uint32_t)G + (uint32_t)__builtin_amdgcn_mbcnt_hi(
                                                          (uint32_t)(mk >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mk, 0u));
            skey[p] = pk;
#pragma unroll
            for (int q = 0; q < NV; ++q)
#pragma unroll
                for (int s = 0; s < G; ++s) sval[(q * G + s) * CAPH + p] = pv[s * NV + q];
        }
        n_staged += (uint32_t)G * (uint32_t)__popcll(mk);
        lds_order();
    }

    // Memory-side addition of one staged value: as is into a fixed-point
    // accumulator, or converted (times inv, the inverse scale) into an FP32 one.
    __device__ static inline void acc_add(unsigned long long* p, unsigned long long x, double) { atomicAdd(p, x); }
    __device__ static inline void acc_add(float* p, unsigned long long x, double inv) {
        unsafeAtomicAdd(p, (float)((double)(long long)x * inv));
    }

    // Converged: as Deposit::flush (kWave / LPE cells, whole groups, per instruction).
    template <class A>
    __device__ inline void flush(A* acc, int lane, uint32_t threshold, double inv) {
        const uint32_t n = n_staged;
        if (n < threshold || n == 0) return;
        const uint32_t per = kWave / LPE;
        const int f = lane % LPE;
        for (uint32_t b0 = 0; b0 < n; b0 += per) {
            const uint32_t e = b0 + (uint32_t)lane / LPE;
            const uint32_t p = e / (uint32_t)G, s = e % (uint32_t)G;
            if (e < n && f < NV)
                acc_add(acc + ((uint64_t)skey[p] * G + s) * LPE + f, sval[(f * G + s) * CAPH + p], inv);
        }
        n_staged = 0u;
        lds_order();
    }

    // Converged: empty the cache into the accumulator.  Fewer than kFlushAt cells
    // may be staged on entry (each pass stages up to G x 64 more).
    template <class A>
    __device__ inline void drain(A* acc, int lane, double inv) {
        for (int s0 = 0; s0 < S; s0 += kWave) {
            const int s = s0 + lane;
            const uint32_t k = keys[s];
            V old[W];
#pragma unroll
            for (int w = 0; w < W; ++w) old[w] = vals[w * S + s];
            stage(k != kEmptyKey, k, old);
            keys[s] = kEmptyKey;
            lds_order();
            flush(acc, lane, 1u, inv);
        }
    }
};

// --------------------------------------------------------------------------
// Forward sweep of one level
// --------------------------------------------------------------------------

// MODE 0: tree only (the tape pass of the adjoint); 1: the rate and the force;
// 2: also J of every bin.  DET: a 64-bit fixed-point accumulator, else FP32 (the
// LDS partial sums are fixed point in both).  The rate is accumulated as what
// Eq. e:photrate2 sums: the gas's share n_HI sigma_H / chi_i of the absorbed
// ionizing luminosity of every segment, so a dense cell's rate is a sum of
// values of the size of the absorbed packets (not a small J times a large n_H).
// Quad pre-combine (DPP lane moves, no LDS): lanes 4k..4k+3 of a wavefront trace
// the four children of one parent pixel and often cross the same cell in the same
// step.  Partners lane^1 and then lane^2 compare keys; on a match the lower lane
// adds the upper lane's values and the upper lane drops its deposit.  Same-address
// LDS atomics serialise, so this removes most of the LDS cache's address and bank
// conflicts for a few VALU instructions.  Converged code (every lane present).
// The values are FP32 (before any fixed-point conversion): one lane move each.
__device__ __forceinline__ uint32_t dpp_u32(uint32_t x, int ctrl) {
    return ctrl == 0xB1 ? (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0xB1, 0xF, 0xF, false)
                        : (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x4E, 0xF, 0xF, false);
}
__device__ __forceinline__ float dpp_v(float x, int ctrl) { return __uint_as_float(dpp_u32(__float_as_uint(x), ctrl)); }
template <int NV>
__device__ __forceinline__ void quad_combine(int lane, uint32_t& key, float (&v)[NV]) {
#pragma unroll
    for (int step = 0; step < 2; ++step) {
        const int ctrl = step == 0 ? 0xB1 : 0x4E;
        const uint32_t kp = dpp_u32(key, ctrl);
        float vp[NV];
#pragma unroll
        for (int q = 0; q < NV; ++q) vp[q] = dpp_v(v[q], ctrl);
        const bool upper = (lane >> step) & 1;
        const bool same = key == kp && key != kEmptyKey;
#pragma unroll
        for (int q = 0; q < NV; ++q) v[q] = (same && !upper) ? v[q] + vp[q] : v[q];
        key = (same && upper) ? kEmptyKey : key;
    }
}

// A wavefront claims 64 consecutive rays of a level with one atomic; lane l
// takes base + l.  The order matters: the quad pre-combine pairs sibling rays
// (four consecutive rays of a level) by lane.  Every lane of the wavefront must
// be present.
// Largest ray pool: pool indices, child links and the per-level claim counters
// are 32-bit, and a counter overshoots its level's end by one 64-ray claim per
// wavefront of the launch (at most 64 workgroups of 4 wavefronts per CU: 2^22
// rays on 256 CUs), so with 2^23 rays of room it never wraps.
constexpr uint64_t kMaxPoolRays = 0xff800000ull;

__device__ __forceinline__ uint32_t claim_rays(uint32_t* head, int lane) {
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(head, (uint32_t)kWave);
    return (uint32_t)__builtin_amdgcn_readlane((int)base, 0) + (uint32_t)lane;
}

// Values per cell and their places in the AoS accumulator (stride 4 or 8):
// MODE 1: rate, F_x, F_y, F_z; MODE 2: J_0, F_x, F_y, F_z, rate[, J_1].
template <int NB, int MODE>
struct SweepVals {
    static constexpr int NV = MODE == 2 ? 4 + NB : 4;
    static constexpr int kRate = MODE == 2 ? 4 : 0;
    static constexpr int kJ1 = 5;
    static constexpr int LPE = NV <= 4 ? 4 : 8;
};
// Forward deposits, both modes: pairs of cells per slot, partial sums in 64-bit
// fixed point in LDS (integer LDS atomics are fast, float ones are not), one
// memory request per evicted pair.  The FP32 mode converts a staged value to
// FP32 at the flush.  9.8 KB of LDS per wavefront: 16 wavefronts fit a CU.
template <int NV>
using SweepDeposit = GroupDeposit<NV, unsigned long long, 2>;
// Adjoint deposits (two values per cell): 256 single-cell slots.  Grouped slots
// (four cells) were slower here: the adjoint is not bound by memory-side atomics.
template <bool DET>
using AdjointDeposit = Deposit<2, typename std::conditional<DET, unsigned long long, double>::type, 256>;

template <int NB, bool DET, int MODE>
// Four wavefronts per SIMD (at most 128 VGPRs): the march is latency bound, and
// the few registers this spills are outside the loop.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) k_sweep(SweepArgs a, int level) {
    using SV = SweepVals<NB, MODE>;
    constexpr int NV = SV::NV;
    using Dep = SweepDeposit<NV>;
    using V = typename Dep::V;
    // Dynamic LDS: Dep::kBytes per wavefront of the workgroup (none in MODE 0)
    extern __shared__ __align__(16) unsigned char sweep_lds[];
    const Geo& g = a.g;
    Counters* ct = a.ct;
    const int lane = lane_id();
    // After a pool overflow the tree is incomplete and some slots were never
    // written: do no further work (the error is reported on synchronisation).
    if (ct->c.status & kStOverflow) return;
    const uint64_t off = ct->w.off[level];
    const uint32_t n_tail = ct->w.tail[level];
    const uint32_t n_level = (uint32_t)std::min<uint64_t>(n_tail, a.pool.cap > off ? a.pool.cap - off : 0);
    const uint64_t off_next = off + n_level;
    const int next = level + 1;
    if (blockIdx.x == 0 && threadIdx.x == 0 && next <= ART_MAX_LEVELS) ct->w.off[next] = off_next;
    const double scale = ct->c.scale;
    const double inv_scale = 1.0 / scale;  // a power of two
    const float lnom_scale = ldexpf(1.0f / 12.0f, -2 * level);  // 1 / N_ray(l)
    const unsigned long long dweight = 1ull << (2 * (g.level_max - level));
    using Acc = typename std::conditional<DET, unsigned long long, float>::type;
    Acc* acc = (Acc*)(DET ? (void*)a.det : (void*)a.acc);

    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    Dep dep = Dep::at(sweep_lds + (MODE ? (size_t)w * Dep::kBytes : 0));
    if (MODE) dep.init(lane);

    auto quant = [&](float x) -> V { return (V)(unsigned long long)fixed_point(x, scale); };

    for (;;) {
        // Every lane claims one ray, and the loop exit is a wave-uniform ballot,
        // so the loop stays a single convergent loop (no lane waits on a value
        // another lane computes under a divergent branch).
        const uint32_t li = claim_rays(&ct->w.head[level], lane);
        const bool active = li < n_level;
        if (__ballot(active) == 0ull) break;
        const uint64_t slot = off + (active ? li : 0u);

        uint32_t src = 0, pix = 0;
        uint32_t nseg = 0;
        double left[NB];
        double tau[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            left[b] = 0.0;
            tau[b] = 0.0;
        }
        bool bad_src = false, stuck = false;
        Ray r;
        MarchState m;
        m.alive = false;
        m.end = kExit;
        float lnom[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) lnom[b] = 0.0f;
        if (active) {
            src = a.pool.src[slot];
            pix = a.pool.pix[slot];
            if (src >= a.n_src) {  // never happens for a written slot; keeps reads in bounds
                bad_src = true;
                src = 0;
            }
#pragma unroll
            for (int b = 0; b < NB; ++b) tau[b] = a.pool.tau[2 * slot + b];
            ray_setup(g, a.src_pos, src, level, pix, r);
#pragma unroll
            for (int b = 0; b < NB; ++b) lnom[b] = a.src_lum[(uint64_t)src * NB + b] * lnom_scale;
            if (bad_src || !source_inside(g, r.xs)) bad_src = true;
            else if (!r.starts_outside) march_begin(g, a.q, r, m, MODE ? a.fg : nullptr);
        }
        // converged march: one segment per lane per iteration
        const float nxf = (float)r.n[0], nyf = (float)r.n[1], nzf = (float)r.n[2];
        // The loop body twice per iteration: the march state then alternates
        // between two register sets instead of being copied back every step.
        auto step = [&]() __attribute__((always_inline)) {
            // the current cell's (n_H, x_n), before march_step moves on
            const float2 qv = m.q;
            if (MODE) {
                // Flush what earlier steps staged, but only after this step's gather
                // has arrived: the vector-memory counter retires in order, so the
                // next step's wait for its gather also waits for these atomics, and
                // issued here they have a whole step to complete.
                __asm__ volatile("" ::"v"(qv.x), "v"(qv.y));
                dep.flush(acc, lane, Dep::kFlushAt, inv_scale);
            }
            // (pk, pv) are read only where deposit() returned true, which assigns them
            bool pend = false;
            uint32_t pk = unset<uint32_t>();
            V pv[Dep::W];
#pragma unroll
            for (int w = 0; w < Dep::W; ++w) pv[w] = unset<V>();
            {
                uint32_t c;
                int ijk[3];
                double dr, dtau[NB], tin[NB];
                const float fgc = m.fg;  // this step's cell, before march_step moves on
                const bool seg =
                    march_step<NB>(g, a.q, r, m, tau, &stuck, c, ijk, dr, dtau, tin, MODE ? a.fg : nullptr);
                if (seg) ++nseg;
                if (MODE) {
                    // without a segment the key below is empty: the quad combine
                    // discards these values and nothing deposits them
                    float v[NV];
#pragma unroll
                    for (int q = 0; q < NV; ++q) v[q] = unset<float>();
                    if (seg) {
#pragma clang fp contract(fast)
                        const float drf = (float)dr;
                        float dLs = 0.0f, dL0 = 0.0f, j0 = 0.0f, j1 = 0.0f;
#pragma unroll
                        for (int b = 0; b < NB; ++b) {
                            const float x = (float)dtau[b];
                            const float Lin = lnom[b] * __expf(-(float)tin[b]);
                            float ph, om;
                            absorb_factors(x, ph, om);
                            const float dL = Lin * om;
                            dLs += dL;
                            if (b == 0) dL0 = dL;
                            if (MODE == 2) {
                                if (b == 0) j0 = Lin * drf * ph;
                                else j1 = Lin * drf * ph;
                            }
                        }
                        // the gas's share of the ionizing bin's absorption (Sec. 2.3
                        // opacities), gathered with the cell's fields
                        v[SV::kRate] = fgc * dL0;
                        v[1] = nxf * dLs;
                        v[2] = nyf * dLs;
                        v[3] = nzf * dLs;
                        if (MODE == 2) {
                            v[0] = j0;
                            if (NB > 1) v[SV::kJ1 % NV] = j1;
                        }
                    }
                    // combined in FP32, then quantised: the pairs are fixed by the
                    // lane order, so fixed-point results stay reproducible
                    uint32_t key = seg ? c : kEmptyKey;
                    quad_combine<NV>(lane, key, v);
                    if (key != kEmptyKey) {
                        V vq[NV];
#pragma unroll
                        for (int q = 0; q < NV; ++q) vq[q] = quant(v[q]);
                        pend = dep.deposit(key, ijk, vq, pk, pv);
                    }
                }
            }
            if (MODE) dep.stage(pend, pk, pv);
        };
        while (__ballot(m.alive)) {
            step();
            if (__ballot(m.alive) == 0ull) break;
            step();
        }
        const int end = m.end;
        if (active && a.pool.last) {
            a.pool.last[slot] = nseg ? m.c : kNoChild;
            a.pool.rlast[slot] = m.rr;
#pragma unroll
            for (int b = 0; b < 2; ++b) a.pool.taulast[2 * slot + b] = b < NB ? tau[b] : 0.0;
        }
        if (active && end != kSplit) {
#pragma unroll
            for (int b = 0; b < NB; ++b)
                left[b] = (double)a.src_lum[(uint64_t)src * NB + b] / (12.0 * ldexp(1.0, 2 * level)) * exp(-tau[b]);
        }
        if (__ballot(bad_src)) {
            if (lane == 0) atomicOr(&ct->c.status, (uint32_t)kStOutside);
        }
        if (__ballot(stuck)) {
            if (lane == 0) atomicOr(&ct->c.status, (uint32_t)kStStuck);
        }

        // ---- children: a splitting ray records the optical depth at the
        //      split; the children are written in parent order afterwards ----
        const bool is_split = active && end == kSplit;
        const bool is_exit = active && end == kExit;
        const bool is_term = active && end == kTerm;
        const uint32_t nsplit = (uint32_t)__popcll(__ballot(is_split));
        if (active) {
            a.pool.tend[2 * slot] = is_split ? tau[0] : -1.0;
            a.pool.tend[2 * slot + 1] = (is_split && NB > 1) ? tau[NB - 1] : 0.0;
        }
        // the claim's 64 rays lie in one tile of the child scan (tiles are whole
        // multiples of a claim): add their splitting rays to its count
        if (lane == 0 && nsplit) atomicAdd(&a.pool.tsum[li / (uint32_t)kSplitTile], nsplit);

        // ---- statistics: one atomic per counter per wavefront when the
        //      chunk belongs to a single source (the common case) ----
        const uint32_t s_first = (uint32_t)__builtin_amdgcn_readfirstlane((int)src);
        const bool mixed = __ballot(active && src != s_first) != 0ull;
        const uint32_t n_act = (uint32_t)__popcll(__ballot(active));
        const uint32_t n_exit = (uint32_t)__popcll(__ballot(is_exit));
        const uint32_t n_term = (uint32_t)__popcll(__ballot(is_term));
        const unsigned long long seg_sum = wave_sum((unsigned long long)nseg);
        if (lane == 0) {
            atomicAdd(&ct->c.destroy, (unsigned long long)(n_exit + n_term) * dweight);
            atomicAdd(&ct->c.segments, seg_sum);
        }
        if (!mixed) {
            double esc[NB], res[NB];
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                esc[b] = wave_sum(is_exit ? left[b] : 0.0);
                res[b] = wave_sum(is_term ? left[b] : 0.0);
            }
            if (lane == 0) {
                const uint64_t sl = (uint64_t)s_first * ART_MAX_LEVELS + level;
                atomicAdd(&a.st.created[sl], n_act);
                if (nsplit) atomicAdd(&a.st.split[sl], nsplit);
                if (n_exit) atomicAdd(&a.st.exited[sl], n_exit);
                if (n_term) atomicAdd(&a.st.term[sl], n_term);
                atomicAdd(&a.st.segments[s_first], seg_sum);
#pragma unroll
                for (int b = 0; b < NB; ++b) {
                    if (n_exit) unsafeAtomicAdd(&a.st.escaped[2 * (uint64_t)s_first + b], esc[b]);
                    if (n_term) unsafeAtomicAdd(&a.st.residual[2 * (uint64_t)s_first + b], res[b]);
                }
            }
        } else if (active) {
            const uint64_t sl = (uint64_t)src * ART_MAX_LEVELS + level;
            atomicAdd(&a.st.created[sl], 1u);
            if (is_split) atomicAdd(&a.st.split[sl], 1u);
            if (is_exit) atomicAdd(&a.st.exited[sl], 1u);
            if (is_term) atomicAdd(&a.st.term[sl], 1u);
            atomicAdd(&a.st.segments[src], (unsigned long long)nseg);
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                if (is_exit) unsafeAtomicAdd(&a.st.escaped[2 * (uint64_t)src + b], left[b]);
                if (is_term) unsafeAtomicAdd(&a.st.residual[2 * (uint64_t)src + b], left[b]);
            }
        }
    }
    if (MODE) {
        dep.flush(acc, lane, 1u, inv_scale);
        dep.drain(acc, lane, inv_scale);
    }
}

// --------------------------------------------------------------------------
// Children of one level, in parent order
// --------------------------------------------------------------------------

// The seed kernel lays out level l0 by source, then by nested pixel.  Writing
// the four children of the k-th splitting parent of a level to places 4k..4k+3
// of the next level keeps every level in that order, so consecutive claims are
// neighbouring directions of one source and the rays in flight at any moment
// cover a small part of the grid (their gathers and deposits stay in cache).
// Per level: the sweep counts the splitting rays of each tile of kSplitTile
// parents as its claims finish; one workgroup turns the counts into exclusive
// prefixes and sets the next level's size; each tile then writes its children
// and clears its count for the next level.
constexpr int kSplitThreads = 256;

// The level's rays [off, off + n); none after a pool overflow, when the tree is
// incomplete and the error is reported on synchronisation.
__device__ inline void level_range(const Pool& pool, const Counters* ct, int level, uint64_t& off, uint32_t& n) {
    off = ct->w.off[level];
    const uint32_t t = ct->w.tail[level];
    n = (uint32_t)std::min<uint64_t>(t, pool.cap > off ? pool.cap - off : 0);
    if (ct->c.status & kStOverflow) n = 0;
}

// One workgroup: exclusive prefix of the tile counts (in place); sets the
// next level's ray count, or the overflow status if the pool cannot hold it.
__global__ void __launch_bounds__(1024) k_split_scan(Pool pool, Counters* ct, int level) {
    __shared__ uint32_t part[1024 / kWave];
    __shared__ uint32_t carry_sh;
    uint64_t off;
    uint32_t n;
    level_range(pool, ct, level, off, n);
    const uint32_t n_tiles = (n + kSplitTile - 1) / kSplitTile;
    const int lane = lane_id(), w = (int)(threadIdx.x >> 6);
    if (threadIdx.x == 0) carry_sh = 0u;
    __syncthreads();
    for (uint32_t b = 0; b < n_tiles; b += blockDim.x) {
        const uint32_t t = b + threadIdx.x;
        const uint32_t v = t < n_tiles ? pool.tsum[t] : 0u;
        uint32_t x = v;  // inclusive scan within the wavefront
        for (int o = 1; o < kWave; o <<= 1) {
            const uint32_t y = __shfl_up(x, o, kWave);
            if (lane >= o) x += y;
        }
        if (lane == kWave - 1) part[w] = x;
        __syncthreads();
        uint32_t before = carry_sh;
        for (int k = 0; k < w; ++k) before += part[k];
        if (t < n_tiles) pool.tsum[t] = before + x - v;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t s = 0;
            for (int k = 0; k < (int)(blockDim.x / kWave); ++k) s += part[k];
            carry_sh += s;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && level + 1 <= ART_MAX_LEVELS) {
        const uint64_t kids = 4ull * carry_sh;
        const uint64_t off_next = off + n;
        if (off_next + kids > pool.cap) atomicOr(&ct->c.status, (uint32_t)kStOverflow);
        ct->w.tail[level + 1] = (uint32_t)std::min<uint64_t>(kids, 0xffffffffull);
    }
}

__global__ void __launch_bounds__(kSplitThreads) k_split_scatter(Pool pool, const Counters* ct, int level) {
    __shared__ uint32_t part[kSplitThreads / kWave];
    uint64_t off;
    uint32_t n;
    level_range(pool, ct, level, off, n);
    const uint64_t off_next = off + n;
    const uint32_t n_tiles = (n + kSplitTile - 1) / kSplitTile;
    const int lane = lane_id(), w = (int)(threadIdx.x >> 6);
    for (uint32_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        uint32_t carry = pool.tsum[t];
        for (uint32_t j0 = 0; j0 < kSplitTile; j0 += kSplitThreads) {
            const uint32_t i = t * kSplitTile + j0 + threadIdx.x;
            const uint64_t s = off + i;
            const bool sp = i < n && pool.tend[2 * s] >= 0.0;
            const unsigned long long m = __ballot(sp);
            if (lane == 0) part[w] = (uint32_t)__popcll(m);
            __syncthreads();
            uint32_t before = carry, all = 0;
            for (int k = 0; k < kSplitThreads / kWave; ++k) {
                if (k < w) before += part[k];
                all += part[k];
            }
            if (sp) {
                const uint32_t r = before + (uint32_t)__builtin_amdgcn_mbcnt_hi(
                                                (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
                const uint64_t cs = off_next + 4ull * r;
                if (cs + 4 <= pool.cap) {
                    const uint32_t src = pool.src[s], pix = pool.pix[s];
                    const double t0 = pool.tend[2 * s], t1 = pool.tend[2 * s + 1];
#pragma unroll
                    for (int k = 0; k < 4; ++k) {
                        pool.src[cs + k] = src;
                        pool.pix[cs + k] = 4u * pix + (uint32_t)k;
                        pool.tau[2 * (cs + k)] = t0;
                        pool.tau[2 * (cs + k) + 1] = t1;
                        if (pool.child) pool.child[cs + k] = kNoChild;
                    }
                    if (pool.child) pool.child[s] = (uint32_t)cs;
                }
            }
            carry += all;
            __syncthreads();
        }
        if (threadIdx.x == 0) pool.tsum[t] = 0u;  // read by every thread above, before the barriers
    }
}

// After the deepest level of a wave: record the number of rays the wave held.
__global__ void k_end_wave(Counters* ct, int level0, int level_max) {
    if (threadIdx.x != 0) return;
    unsigned long long tot = 0;
    for (int l = level0; l <= level_max + 1 && l <= ART_MAX_LEVELS; ++l) tot += ct->w.tail[l];
    atomicMax(&ct->c.rays_wave_max, tot);
}

// rate (accumulated as the gas's share of the absorbed ionizing luminosity,
// Eq. e:photrate2), force and J from the AoS accumulator (stride lpe: 4 without
// J, 8 with J), unpacking fixed point in deterministic mode.  Transparent cells
// get no rate or force (nothing is absorbed there).
template <bool DET>
__global__ void k_finalize(uint64_t N, const uint8_t* transparent, const float* acc, const unsigned long long* det,
                           int lpe, const Counters* ct, float* rate, float* force, float* J, int n_bins) {
    const double inv = DET ? ct->c.inv_scale : 0.0;
    const int f_rate = lpe == 8 ? 4 : 0;
    for (uint64_t c = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; c < N;
         c += (uint64_t)gridDim.x * blockDim.x) {
        double v[6];
#pragma unroll
        for (int f = 0; f < 6; ++f) {
            if (f >= 4 && (lpe < 8 || f >= 4 + n_bins)) {
                v[f] = 0.0;
                continue;
            }
            v[f] = DET ? (double)(long long)det[c * lpe + f] * inv : (double)acc[c * lpe + f];
        }
        const bool sink = transparent && transparent[c];
        rate[c] = sink ? 0.0f : (float)v[f_rate];
        force[c] = sink ? 0.0f : (float)v[1];
        force[N + c] = sink ? 0.0f : (float)v[2];
        force[2 * N + c] = sink ? 0.0f : (float)v[3];
        if (J && lpe == 8) {
            J[c] = (float)v[0];
            if (n_bins > 1) J[N + c] = (float)v[5];
        }
    }
}

// --------------------------------------------------------------------------
// Adjoint sweep of one level (children first: launched from the deepest level)
// --------------------------------------------------------------------------


// For every ray of the level, its segments are walked once, backwards (from the
// tape's last cell to the ray's start), depositing dL/dkappa_b of each crossed
// cell:
//   [b = ionizing] a L_in dr^2 phi'(dtau) + beta L_in dr e^{-dtau} - dr G_b(after the segment)
// with a = w s_H x_n n_H (the rate weight) and beta = v . n (the force weight):
// every downstream contribution is proportional to e^{-tau}, so its derivative
// with respect to this segment's opacity is -dr times its value.  Walking
// backwards, G_b(after) is the children's G_b(start) plus the ray's own loss
// terms of the segments already walked; at the start it is G_b(start), stored
// for the parent level.  L_in = L_nom e^{-tau_in} comes from the end's optical
// depth (tape) by removing each segment's dtau.  The segments are those of the
// forward walk (same expressions), and the tree is the forward's.  The gradient
// of a cell is a sum of terms of both signs, so the per-segment arithmetic is
// FP64 and the two values per cell go through the same LDS cache as the
// forward deposits, as FP64 or as 64-bit fixed point.
template <int NB, bool DET>
// Three wavefronts per SIMD (at most 168 VGPRs); the registers this spills are
// outside the walk loop.
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) k_adjoint(AdjArgs a, int level) {
    using V = typename std::conditional<DET, unsigned long long, double>::type;
    using Dep = AdjointDeposit<DET>;
    extern __shared__ __align__(16) unsigned char adj_lds[];
    const Geo& g = a.g;
    Counters* ct = a.ct;
    if (ct->c.status & kStOverflow) return;
    const int lane = lane_id();
    const uint64_t off = ct->w.off[level];
    const uint32_t n_level =
        (uint32_t)std::min<uint64_t>(ct->w.tail[level], a.pool.cap > off ? a.pool.cap - off : 0);
    const double gscale_n = DET ? ct->c.gscale[0] : 0.0, gscale_x = DET ? ct->c.gscale[1] : 0.0;
    const double inv_nray = 1.0 / (12.0 * ldexp(1.0, 2 * level));
    const double sH = g.s_H, sd = g.s_d;
    V* acc = (V*)(DET ? (void*)a.gdet : (void*)a.gk);
    const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    Dep dep = Dep::at(adj_lds + (size_t)w * Dep::kBytes);
    dep.init(lane);
    auto quant = [&](double x, double gscale) -> V {
        if (DET) return (V)(unsigned long long)__double2ll_rn(x * gscale);
        else return (V)x;
    };

    for (;;) {
        const uint32_t li = claim_rays(&ct->w.adj_head[level], lane);
        const bool active = li < n_level;
        if (__ballot(active) == 0ull) break;
        const uint64_t slot = off + (active ? li : 0u);

        uint32_t src = 0, pix = 0, last = kNoChild;
        double tau[NB], E[NB], lnom[NB], Gend[NB], A[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            tau[b] = 0.0;
            E[b] = 1.0;
            lnom[b] = 0.0;
            Gend[b] = 0.0;
            A[b] = 0.0;
        }
        bool run = false, stuck = false;
        Ray r;
        BackState m;
        m.alive = false;
        if (active) {
            src = a.pool.src[slot];
            pix = a.pool.pix[slot];
            last = a.pool.last[slot];
            const bool ok = src < a.n_src;  // always true for a written slot
            if (!ok) src = 0;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                tau[b] = a.pool.taulast[2 * slot + b];
                E[b] = exp(-tau[b]);
                lnom[b] = (double)a.src_lum[(uint64_t)src * NB + b] * inv_nray;
            }
            const uint32_t ch = a.pool.child[slot];
            if (ch != kNoChild) {
                for (int k = 0; k < 4; ++k)
#pragma unroll
                    for (int b = 0; b < NB; ++b) Gend[b] += a.pool.G[2 * ((uint64_t)ch + k) + b];
            }
            ray_setup(g, a.src_pos, src, level, pix, r);
            run = ok && last != kNoChild && source_inside(g, r.xs) && !r.starts_outside;
            if (run) back_begin(g, a.q, r, last, a.pool.rlast[slot], m);
        }
        const double nx = r.n[0], ny = r.n[1], nz = r.n[2];

        // two steps per iteration, as in the forward sweep
        auto step = [&]() __attribute__((always_inline)) {
            bool pend = false;
            uint32_t pk = 0;
            V pv[Dep::W];
            {
                uint32_t c;
                int ijk[3];
                double dr, dtau[NB];
                const float2 qc = m.q;
                // as in the forward sweep: flush once this step's gather has arrived,
                // so the atomics are not waited for by the loads that follow at once
                __asm__ volatile("" ::"v"(qc.x), "v"(qc.y));
                dep.flush(acc, lane, Dep::kFlushAt);
                const bool seg = back_step<NB>(g, a.q, r, m, &stuck, c, ijk, dr, dtau);
                V v[2] = {(V)0, (V)0};
                if (seg) {
                    const float4 wv = a.wv[c];
                    const double xv = (double)qc.y, nv = (double)qc.x;
                    const double wa = (double)wv.x * sH * xv * nv;
                    const double beta = (double)wv.y * nx + (double)wv.z * ny + (double)wv.w * nz;
                    double dkap[NB], j0 = 0.0;
#pragma unroll
                    for (int b = 0; b < NB; ++b) {
                        const double x = dtau[b];
                        double e, om;
                        double einv;
                        exp_neg_pos(x, e, om, einv);
                        // transmission at the segment's entry: E(out) e^{+dtau}, or
                        // directly where either underflows
                        tau[b] -= min_f64(x, kTauStep);
                        double Ein = E[b] * einv;
                        if (!(E[b] > 1e-290 && e > 1e-290)) Ein = exp(-tau[b]);
                        E[b] = Ein;
                        const double Lin = lnom[b] * Ein;
                        double own = beta * Lin * om;
                        double dk = beta * Lin * dr * e;
                        if (b == 0) {
                            double ph, dph;
                            absorb_phi_dphi(x, e, om, ph, dph);
                            j0 = Lin * dr * ph;
                            own += wa * j0;
                            dk += wa * Lin * dr * dr * dph;
                        }
                        dkap[b] = dk - dr * (A[b] + Gend[b]);
                        A[b] += own;
                    }
                    // chain rule through kappa_0 = n_H (x_n s_H + s_d), kappa_1 = n_H s_d,
                    // plus the explicit n_H x_n factor of rate = s_H x_n n_H J_0
                    const double wj = (double)wv.x * sH * j0;
                    double gn = dkap[0] * (xv * sH + sd) + wj * xv;
                    if (NB > 1) gn += dkap[NB - 1] * sd;
                    const double gx = dkap[0] * nv * sH + wj * nv;
                    v[0] = quant(gn, gscale_n);
                    v[1] = quant(gx, gscale_x);
                }
                if (seg) pend = dep.deposit(c, ijk, v, pk, pv);
            }
            dep.stage(pend, pk, pv);
        };
        while (__ballot(m.alive)) {
            step();
            if (__ballot(m.alive) == 0ull) break;
            step();
        }
        if (__ballot(stuck)) {
            if (lane == 0) atomicOr(&ct->c.status, (uint32_t)kStStuck);
        }
        if (active) {
#pragma unroll
            for (int b = 0; b < NB; ++b) a.pool.G[2 * slot + b] = A[b] + Gend[b];
        }
    }
    dep.flush(acc, lane, 1u);
    dep.drain(acc, lane);
}

// Clear the adjoint's per-level claim counters (a reused tree is walked again).
__global__ void k_adj_reset(Counters* ct) {
    if (blockIdx.x == 0 && threadIdx.x <= ART_MAX_LEVELS) ct->w.adj_head[threadIdx.x] = 0u;
}

template <int NB, bool DET>
size_t adjoint_lds_bytes(unsigned block) {
    return (size_t)(block / kWave) * AdjointDeposit<DET>::kBytes;
}

// Convert the accumulated dL/dn_H and dL/dx_n to the FP32 outputs.
template <bool DET>
__global__ void k_adj_finalize(uint64_t N, const double* gk, const unsigned long long* gdet, const Counters* ct,
                               const uint8_t* transparent, float* g_nH, float* g_xn) {
    const double ginv_n = DET ? ct->c.inv_gscale[0] : 0.0, ginv_x = DET ? ct->c.inv_gscale[1] : 0.0;
    for (uint64_t c = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; c < N;
         c += (uint64_t)gridDim.x * blockDim.x) {
        if (transparent && transparent[c]) {  // the outputs do not depend on these fields
            g_nH[c] = 0.0f;
            g_xn[c] = 0.0f;
        } else if (DET) {
            g_nH[c] = (float)((double)(long long)gdet[2 * c] * ginv_n);
            g_xn[c] = (float)((double)(long long)gdet[2 * c + 1] * ginv_x);
        } else {
            g_nH[c] = (float)gk[2 * c];
            g_xn[c] = (float)gk[2 * c + 1];
        }
    }
}

// --------------------------------------------------------------------------
// Ionization subcycle (Sec. 2.3): substep size and Method B update
// --------------------------------------------------------------------------

// ion[0]: min over cells of n_H / |I - R| as the bits of a non-negative double
// (such bit patterns order like the values, so an unsigned atomic min works);
// ion[1]: the substep's dt (bits); ion[2]: time of art_ion_subcycle's own clock.
__global__ void k_ion_begin(unsigned long long* ion) {
    if (threadIdx.x == 0 && blockIdx.x == 0) ion[0] = 0x7ff0000000000000ull;  // +inf
}

__global__ void __launch_bounds__(256) k_ion_minq(uint64_t N, const float* nH, const float* xn, const float* J0,
                                                  const uint8_t* transparent, double gamma_scale, double alpha_B,
                                                  unsigned long long* ion) {
    __shared__ double part[256 / kWave];
    double q = INFINITY;
    for (uint64_t c = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; c < N; c += (uint64_t)gridDim.x * blockDim.x) {
        const double n = (double)nH[c];
        if (!(n > 0.0) || (transparent && transparent[c])) continue;
        const double x = (double)xn[c];
        const double ne = n * (1.0 - x);
        const double I = gamma_scale * (double)J0[c] * n * x;
        const double R = alpha_B * ne * ne;
        const double d = fabs(I - R);
        if (d > 0.0) q = fmin(q, n / d);
    }
    for (int o = kWave / 2; o > 0; o >>= 1) q = fmin(q, __shfl_xor(q, o, kWave));
    if (lane_id() == 0) part[threadIdx.x >> 6] = q;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < (int)(blockDim.x / kWave); ++k) q = fmin(q, part[k]);
        // Same-address atomics serialise; the running minimum only decreases, so a
        // block whose value is not below a (possibly stale) read of it can skip its
        // atomic.  Non-negative doubles order like their bit patterns.
        const unsigned long long qb = (unsigned long long)__double_as_longlong(q);
        if (qb < __hip_atomic_load(&ion[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMin(&ion[0], qb);
    }
}

__global__ void k_ion_dt(unsigned long long* ion, double C, double t_end, double* t_now) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double q = __longlong_as_double((long long)ion[0]);
    const double t = *t_now;
    const double rem = t_end - t;
    double dt = C * q;  // +inf if no cell changes
    const bool last = !(dt < rem);
    if (last) dt = rem;
    if (!(dt > 0.0)) dt = 0.0;
    ion[1] = (unsigned long long)__double_as_longlong(dt);
    *t_now = (last && rem > 0.0) ? t_end : t + dt;
}

__global__ void k_ion_update(uint64_t N, const float* nH, float* xn, const float* J0, const float* force,
                             const uint8_t* transparent, float* impulse, double gamma_scale, double alpha_B,
                             const unsigned long long* ion) {
    const double dt = __longlong_as_double((long long)ion[1]);
    if (!(dt > 0.0)) return;
    for (uint64_t c = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; c < N; c += (uint64_t)gridDim.x * blockDim.x) {
        if (transparent && transparent[c]) continue;  // sink cells keep their ionization state
        const double x0 = (double)xn[c];
        const double a = alpha_B * (double)nH[c] * (1.0 - x0);
        const double s = gamma_scale * (double)J0[c] + a;
        if (s > 0.0) {
            const double xeq = a / s;
            xn[c] = (float)(xeq + (x0 - xeq) * exp(-dt * s));
        }
        if (impulse) {
#pragma unroll
            for (int k = 0; k < 3; ++k)
                impulse[k * N + c] = (float)((double)impulse[k * N + c] + (double)force[k * N + c] * dt);
        }
    }
}

// --------------------------------------------------------------------------
// Rotation of the ray directions (Sec. 2.1: random at every time step)
// --------------------------------------------------------------------------

struct Mat3 {
    double m[9];
};

__global__ void k_set_rot(Mat3 r, double* rot) {
    if (threadIdx.x < 9 && blockIdx.x == 0) rot[threadIdx.x] = r.m[threadIdx.x];
}

// Uniform (Haar) random rotation from three uniform numbers (Shoemake's
// quaternion construction): q = (sqrt(1-u1) sin 2pi u2, sqrt(1-u1) cos 2pi u2,
// sqrt(u1) sin 2pi u3, sqrt(u1) cos 2pi u3) = (x, y, z, w) and its matrix.
__global__ void k_random_rot(const double* u, double* rot) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const double u1 = u[0], a = sqrt(1.0 - u1), b = sqrt(u1);
    double s2, c2, s3, c3;
    sincos(2.0 * M_PI * u[1], &s2, &c2);
    sincos(2.0 * M_PI * u[2], &s3, &c3);
    const double x = a * s2, y = a * c2, z = b * s3, w = b * c3;
    rot[0] = 1.0 - 2.0 * (y * y + z * z);
    rot[1] = 2.0 * (x * y - z * w);
    rot[2] = 2.0 * (x * z + y * w);
    rot[3] = 2.0 * (x * y + z * w);
    rot[4] = 1.0 - 2.0 * (x * x + z * z);
    rot[5] = 2.0 * (y * z - x * w);
    rot[6] = 2.0 * (x * z - y * w);
    rot[7] = 2.0 * (y * z + x * w);
    rot[8] = 1.0 - 2.0 * (x * x + y * y);
}

}  // namespace

// --------------------------------------------------------------------------
// Host side
// --------------------------------------------------------------------------

struct art_ctx {
    int nx, ny, nz;
    uint64_t N;
    art_params p;
    art_options o;
    hipStream_t stream;
    int device;
    int cu_count;
    Geo geo;
    Pool pool;
    uint64_t per_src_bound;
    int wave_max;               // sources the pool holds in one wave
    int wave_cap = 0;           // at most this many sources per wave (0: wave_max)
    double* dirs = nullptr;     // [3 * kDirTable] HEALPix centres of the coarse levels (wave planning)
    unsigned long long* sbound = nullptr;  // [max_sources] rays bound per source of the last planned call
    int* wtab = nullptr;        // [max_sources + 2] first source of each planned wave
    bool last_planned = false;  // the last call planned its waves on the device
    int adj_block = 64;         // launch shape of the adjoint sweeps
    int adj_bpc = 16;
    int cur_wave = 1;           // sources in the wave being swept (sizes the shallow levels' grids)
    int deepest;                // deepest level that can hold rays in this grid
    Counters* ct;
    SrcStats st;
    float* acc;              // [8][N] AoS deposit accumulator (atomic mode)
    unsigned long long* det; // [8][N] the same in fixed point (deterministic mode)
    double* gk;
    unsigned long long* gdet;
    float* fscratch;
    unsigned long long* ion;  // [4] ionization subcycle: min n_H/|I-R| bits, dt bits, own clock
    double* rot;              // [9] rotation of the ray directions read by the sweeps
    const uint8_t* transparent = nullptr;  // caller's per-cell sink flags, or none
    float2* q;                // [N] packed (n_H, x_n)
    float* fg;                // [N] gas share of the ionizing opacity
    float4* wv;               // [N] packed adjoint weights (w, v_x, v_y, v_z)
    int n_shell;                // levels whose radial shells one cell can meet (fixed-point bound)
    // tape of the last forward: its tree stays in the pool (single-wave traces only)
    // until a later call overwrites the pool or changes what the tree depends on
    const void* tape_key[4];
    int tape_nsrc;
    bool tape_ok;
    uint64_t tape_gen;          // token of the valid tape (0: none)
    uint64_t gen;               // forward calls so far
    int last_nsrc, last_waves;
    // timing
    bool timing;
    std::vector<hipEvent_t> ev;
    int ev_used;
    hipEvent_t ev_call0, ev_call1;
};

namespace {

#define HIP_TRY(x)                                        \
    do {                                                  \
        hipError_t e_ = (x);                              \
        if (e_ != hipSuccess) return ART_ERR_HIP;         \
    } while (0)

int fill_blocks(uint64_t n) {
    uint64_t b = (n + 255) / 256;
    if (b > 4096) b = 4096;
    if (b < 1) b = 1;
    return (int)b;
}

template <class T>
int zero(art_ctx* c, T* p, uint64_t n);
template <>
int zero<float>(art_ctx* c, float* p, uint64_t n) {
    if (!n) return ART_OK;
    hipLaunchKernelGGL(k_fill_f32, dim3(fill_blocks(n)), dim3(256), 0, c->stream, p, n);
    HIP_TRY(hipGetLastError());
    return ART_OK;
}
template <>
int zero<double>(art_ctx* c, double* p, uint64_t n) {
    if (!n) return ART_OK;
    hipLaunchKernelGGL(k_fill_f64, dim3(fill_blocks(n)), dim3(256), 0, c->stream, p, n);
    HIP_TRY(hipGetLastError());
    return ART_OK;
}
template <>
int zero<unsigned long long>(art_ctx* c, unsigned long long* p, uint64_t n) {
    if (!n) return ART_OK;
    hipLaunchKernelGGL(k_fill_u64, dim3(fill_blocks(n)), dim3(256), 0, c->stream, p, n);
    HIP_TRY(hipGetLastError());
    return ART_OK;
}
template <>
int zero<uint32_t>(art_ctx* c, uint32_t* p, uint64_t n) {
    if (!n) return ART_OK;
    hipLaunchKernelGGL(k_fill_u32, dim3(fill_blocks(n)), dim3(256), 0, c->stream, p, n, 0u);
    HIP_TRY(hipGetLastError());
    return ART_OK;
}
// The per-source counters of ms sources (levels, bins, segments).
int zero_stats(art_ctx* c, uint64_t ms) {
    hipLaunchKernelGGL(k_zero_stats, dim3(fill_blocks(ms * ART_MAX_LEVELS)), dim3(256), 0, c->stream, c->st, ms);
    HIP_TRY(hipGetLastError());
    return ART_OK;
}

double r_max_host(double phi_c, int level) { return sqrt(3.0 / (M_PI * phi_c)) * ldexp(1.0, level); }

// Upper bound on the rays one source can create at each level, from geometry
// alone: level-l rays exist only where r_max(l-1) is inside the box, and the
// parents that split at r_max(l-1) have pixel centres on the part of that
// sphere inside the box, whose area is at most the box surface S; each such
// pixel covers 1/m_ray of area there, so at most ~4 m_ray S children (a factor
// 2 of margin for pixels straddling the boundary).
uint64_t rays_bound_per_source(int nx, int ny, int nz, const art_params& p) {
    const double diag = sqrt((double)nx * nx + (double)ny * ny + (double)nz * nz);
    const double S = 2.0 * ((double)nx * ny + (double)ny * nz + (double)nz * nx);
    uint64_t tot = 0;
    for (int l = p.level0; l <= p.level_max; ++l) {
        const uint64_t all = 12ull << (2 * l);
        if (l == p.level0) {
            tot += all;
            continue;
        }
        if (r_max_host(p.phi_c, l - 1) >= diag) break;
        const double geo = 4.0 * (2.0 * p.phi_c * S + 1024.0);
        tot += (uint64_t)std::min((double)all, geo);
    }
    return tot;
}

// Level l holds rays only if its parents could split, i.e. if r_max(l-1) is
// below the largest distance from a source inside the box to a point of it (at
// most the box diagonal); deeper levels stay empty and are not launched.
int deepest_level(int nx, int ny, int nz, const art_params& p) {
    const double diag = sqrt((double)nx * nx + (double)ny * ny + (double)nz * nz);
    int l = p.level0;
    while (l < p.level_max && r_max_host(p.phi_c, l) < diag) ++l;
    return l;
}

// Levels whose radial shells [r_a(l), r_max(l)] a cell can meet: a cell spans at
// most sqrt(3) in distance from a source, so it meets the two shells at the ends
// of that range and every shell in between, each no wider than sqrt(3).
int shells_per_cell(const art_params& p) {
    int n = 2;
    for (int l = p.level0; l < p.level_max; ++l) {
        const double width = l == p.level0 ? r_max_host(p.phi_c, l) : r_max_host(p.phi_c, l - 1);
        if (width <= sqrt(3.0)) ++n;
    }
    return n;
}

// Grid, method constants and the tree's size bounds of a context.
void init_geometry(art_ctx* c, int nx, int ny, int nz, const art_params& p) {
    Geo& g = c->geo;
    g.nx = nx;
    g.ny = ny;
    g.nz = nz;
    g.level0 = p.level0;
    g.level_max = p.level_max;
    g.n_bins = p.n_bins;
    g.tau_term = p.tau_term;
    g.s_H = p.s_H;
    g.s_d = p.s_d;
    g.rot = nullptr;  // set once the device copy exists
    for (int l = 0; l < ART_MAX_LEVELS; ++l) g.rmax[l] = r_max_host(p.phi_c, l);
    c->per_src_bound = rays_bound_per_source(nx, ny, nz, p);
    c->deepest = deepest_level(nx, ny, nz, p);
    c->n_shell = shells_per_cell(p);
}

int check_params(const art_params* p) {
    if (!p) return ART_ERR_INVALID_ARG;
    if (p->level0 < 0 || p->level_max < p->level0 || p->level_max >= ART_MAX_LEVELS) return ART_ERR_INVALID_ARG;
    if (p->level_max > 14) return ART_ERR_INVALID_ARG;  // 12*4^l pixel ids must fit 32 bits
    if (p->n_bins < 1 || p->n_bins > ART_MAX_BINS) return ART_ERR_INVALID_ARG;
    if (!(p->phi_c > 0.0) || !(p->tau_term > 0.0) || !(p->tau_term < 0.5 * kTauStep) || !(p->s_H >= 0.0) ||
        !(p->s_d >= 0.0))
        return ART_ERR_INVALID_ARG;
    if (p->deposit_mode != ART_DEPOSIT_ATOMIC && p->deposit_mode != ART_DEPOSIT_DETERMINISTIC)
        return ART_ERR_INVALID_ARG;
    for (int i = 0; i < 9; ++i)
        if (!isfinite(p->rot[i])) return ART_ERR_INVALID_ARG;
    return ART_OK;
}

void free_all(art_ctx* c) {
    (void)hipFree(c->pool.src);
    (void)hipFree(c->pool.pix);
    (void)hipFree(c->pool.tau);
    (void)hipFree(c->pool.child);
    (void)hipFree(c->pool.last);
    (void)hipFree(c->pool.rlast);
    (void)hipFree(c->pool.taulast);
    (void)hipFree(c->pool.tend);
    (void)hipFree(c->pool.tsum);
    (void)hipFree(c->ct);
    (void)hipFree(c->st.created);
    (void)hipFree(c->st.split);
    (void)hipFree(c->st.exited);
    (void)hipFree(c->st.term);
    (void)hipFree(c->st.escaped);
    (void)hipFree(c->st.residual);
    (void)hipFree(c->st.segments);
    (void)hipFree(c->acc);
    (void)hipFree(c->det);
    (void)hipFree(c->gk);
    (void)hipFree(c->gdet);
    (void)hipFree(c->fscratch);
    (void)hipFree(c->ion);
    (void)hipFree(c->rot);
    (void)hipFree(c->q);
    (void)hipFree(c->fg);
    (void)hipFree(c->dirs);
    (void)hipFree(c->sbound);
    (void)hipFree(c->wtab);
    (void)hipFree(c->wv);
    for (hipEvent_t e : c->ev) (void)hipEventDestroy(e);
    if (c->ev_call0) (void)hipEventDestroy(c->ev_call0);
    if (c->ev_call1) (void)hipEventDestroy(c->ev_call1);
}

template <class T>
bool dmalloc(T** p, uint64_t n) {
    *p = nullptr;
    if (n == 0) return true;
    return hipMalloc((void**)p, n * sizeof(T)) == hipSuccess;
}

SweepArgs sweep_args(art_ctx* c, const float* nH, const float* xn, const double* pos, const float* lum,
                     float* force, float* J, int n_src) {
    SweepArgs a;
    a.g = c->geo;
    a.q = c->q;
    a.fg = c->fg;
    a.nH = nH;
    a.xn = xn;
    a.src_pos = pos;
    a.src_lum = lum;
    a.pool = c->pool;
    a.ct = c->ct;
    a.st = c->st;
    a.acc = c->acc;
    (void)force;
    (void)J;
    a.det = c->det;
    a.N = (uint32_t)c->N;
    a.n_src = (uint32_t)n_src;
    return a;
}

// mode 0: tree only (adjoint tape pass); 1: rate + force; 2: rate + force + J
template <int NB, int MODE>
size_t sweep_lds_bytes(unsigned block) {
    return MODE ? (size_t)(block / kWave) * SweepDeposit<SweepVals<NB, MODE>::NV>::kBytes : 0;
}

// At most n_wave * 12 * 4^l rays exist at level l (and no more than the pool
// holds): shallow levels of a few sources get a grid that fits their rays
// instead of the full resident grid, whose idle workgroups would only add
// launch time.
uint64_t level_rays_bound(const art_ctx* c, int level) {
    const uint64_t all = (12ull << (2 * level)) * (uint64_t)std::max(1, c->cur_wave);
    return std::min<uint64_t>(all, c->pool.cap);
}

unsigned level_blocks(const art_ctx* c, int level, int block, int per_cu) {
    const uint64_t full = (uint64_t)c->cu_count * (uint64_t)per_cu;
    const uint64_t need = (level_rays_bound(c, level) + block - 1) / block;
    return (unsigned)std::max<uint64_t>(1, std::min(full, need));
}

// Sources per wave: what the pool holds, or the tuned cap if smaller.
int wave_len(const art_ctx* c) { return c->wave_cap > 0 ? std::min(c->wave_cap, c->wave_max) : c->wave_max; }

int launch_sweep(art_ctx* c, const SweepArgs& a, int level, int mode) {
    const dim3 grid(level_blocks(c, level, c->o.block_size, c->o.blocks_per_cu)), block((unsigned)c->o.block_size);
    const bool det = c->p.deposit_mode == ART_DEPOSIT_DETERMINISTIC;
    const int nb = c->p.n_bins;
    const bool tm = c->timing && c->ev_used + 2 <= (int)c->ev.size();
    if (tm) HIP_TRY(hipEventRecord(c->ev[c->ev_used], c->stream));
#define SWEEP(NB, DET, MODE)                                                                      \
    hipLaunchKernelGGL((k_sweep<NB, DET, MODE>), grid, block, (sweep_lds_bytes<NB, MODE>(block.x)), c->stream, a, \
                       level)
#define SWEEP_MODES(NB, DET)                \
    do {                                    \
        if (mode == 2) SWEEP(NB, DET, 2);   \
        else if (mode == 1) SWEEP(NB, DET, 1); \
        else SWEEP(NB, DET, 0);             \
    } while (0)
    if (nb == 1) {
        if (det) SWEEP_MODES(1, true);
        else SWEEP_MODES(1, false);
    } else if (det) {
        SWEEP_MODES(2, true);
    } else {
        SWEEP_MODES(2, false);
    }
#undef SWEEP_MODES
#undef SWEEP
    HIP_TRY(hipGetLastError());
    if (tm) {
        HIP_TRY(hipEventRecord(c->ev[c->ev_used + 1], c->stream));
        c->ev_used += 2;
    }
    return ART_OK;
}

int launch_adjoint(art_ctx* c, const AdjArgs& a, int level) {
    const dim3 grid(level_blocks(c, level, c->adj_block, c->adj_bpc)), block((unsigned)c->adj_block);
    const bool det = c->p.deposit_mode == ART_DEPOSIT_DETERMINISTIC;
    const size_t lds = det ? adjoint_lds_bytes<1, true>(block.x) : adjoint_lds_bytes<1, false>(block.x);
    if (c->p.n_bins == 1) {
        if (det) hipLaunchKernelGGL((k_adjoint<1, true>), grid, block, lds, c->stream, a, level);
        else hipLaunchKernelGGL((k_adjoint<1, false>), grid, block, lds, c->stream, a, level);
    } else {
        if (det) hipLaunchKernelGGL((k_adjoint<2, true>), grid, block, lds, c->stream, a, level);
        else hipLaunchKernelGGL((k_adjoint<2, false>), grid, block, lds, c->stream, a, level);
    }
    HIP_TRY(hipGetLastError());
    return ART_OK;
}

// Seed wave w: sources s0 .. s0 + n_wave - 1, or (planned) those of the device's
// wave table, of which n_wave is then an upper bound.
int seed_wave(art_ctx* c, int s0, int n_wave, bool planned, int w) {
    c->cur_wave = n_wave;
    const uint64_t n = (uint64_t)(12ull << (2 * c->p.level0)) * (uint64_t)n_wave;
    hipLaunchKernelGGL(k_seed, dim3(fill_blocks(n)), dim3(256), 0, c->stream, c->pool, c->ct, c->p.level0, s0,
                       n_wave, planned ? (const int*)c->wtab : nullptr, w, c->pool.child ? 1 : 0);
    HIP_TRY(hipGetLastError());
    return ART_OK;
}

// Source waves of a call: as many sources per wave as the pool holds for the
// geometric bound every source shares (or the tuned cap), or, when that takes
// more than one wave, waves planned on the device from each source's own bound
// (no host synchronisation: the host launches the fixed-size plan's number of
// waves, and those the device plan does not need find no rays).  per_wave()
// sweeps one seeded wave.  Returns the number of waves launched.
template <class F>
int for_waves(art_ctx* c, const double* src_pos, int n_src, int* launched, F&& per_wave) {
    const int len = wave_len(c);
    const int W = n_src > 0 ? (n_src + len - 1) / len : 0;
    const bool plan = W > 1 && c->wave_cap == 0 && c->dirs;
    c->last_planned = plan;
    if (plan) {
        const unsigned long long loose = c->per_src_bound;
        hipLaunchKernelGGL(k_src_bound, dim3(n_src), dim3(256), 0, c->stream, c->geo, src_pos, n_src, c->dirs,
                           c->deepest, loose, c->sbound);
        hipLaunchKernelGGL(k_plan_waves, dim3(1), dim3(64), 0, c->stream, (const unsigned long long*)c->sbound,
                           n_src, (unsigned long long)c->pool.cap, W, c->wtab);
        HIP_TRY(hipGetLastError());
    }
    for (int w = 0; w < W; ++w) {
        const int s0 = w * len;
        const int nw = plan ? n_src : std::min(len, n_src - s0);
        int rc = seed_wave(c, s0, nw, plan, w);
        if (rc) return rc;
        if ((rc = per_wave())) return rc;
    }
    *launched = W;
    return ART_OK;
}

// Sweep every level of the current wave, l0 first.
// Children of level l, in parent order (the sweep of level l counted them per tile).
int split_level(art_ctx* c, int l) {
    const uint64_t tiles = (level_rays_bound(c, l) + kSplitTile - 1) / kSplitTile;
    const int blocks = (int)std::max<uint64_t>(1, std::min<uint64_t>(4096, tiles));
    hipLaunchKernelGGL(k_split_scan, dim3(1), dim3(1024), 0, c->stream, c->pool, c->ct, l);
    hipLaunchKernelGGL(k_split_scatter, dim3(blocks), dim3(kSplitThreads), 0, c->stream, c->pool, c->ct, l);
    HIP_TRY(hipGetLastError());
    return ART_OK;
}

int sweep_wave(art_ctx* c, const SweepArgs& a, int mode) {
    for (int l = c->p.level0; l <= c->deepest; ++l) {
        int rc = launch_sweep(c, a, l, mode);
        if (rc) return rc;
        if (l < c->deepest && (rc = split_level(c, l))) return rc;
    }
    hipLaunchKernelGGL(k_end_wave, dim3(1), dim3(64), 0, c->stream, c->ct, c->p.level0, c->p.level_max);
    HIP_TRY(hipGetLastError());
    return ART_OK;
}

int begin_call(art_ctx* c, const float* lum, int n_src, const float* nH, const float* xn) {
    hipLaunchKernelGGL(k_begin_call, dim3(1), dim3(256), 0, c->stream, c->ct, lum, n_src, c->p.n_bins, c->p.level0,
                       c->n_shell);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_pack, dim3(fill_blocks(c->N)), dim3(256), 0, c->stream, c->N, nH, xn, c->transparent,
                       c->q, c->fg, c->p.s_H, c->p.s_d, c->ct);
    HIP_TRY(hipGetLastError());
    return ART_OK;
}

}  // namespace

extern "C" {

const char* art_strerror(int code) {
    switch (code) {
        case ART_OK: return "ok";
        case ART_ERR_INVALID_ARG: return "invalid argument";
        case ART_ERR_HIP: return "HIP runtime error";
        case ART_ERR_OUT_OF_MEMORY: return "out of device memory for the workspace";
        case ART_ERR_QUEUE_OVERFLOW: return "ray pool overflow (increase pool_rays)";
        case ART_ERR_SOURCE_OUTSIDE: return "a source lies outside the domain";
        case ART_ERR_DESTROY_COUNT: return "destroy counter does not match N_src*12*4^level_max";
        case ART_ERR_NO_FORWARD: return "no forward tape matches this adjoint call";
        case ART_ERR_NO_ADJOINT: return "context was created without adjoint support";
        case ART_ERR_TOO_LARGE: return "grid and sources exceed the static workspace of art_trace_noalloc";
        case ART_ERR_BAD_FIELD: return "a cell has n_H < 0 or not finite, or x_n outside [0, 1]";
        default: return "unknown error";
    }
}

int art_create(art_ctx** out, int nx, int ny, int nz, const art_params* params, const art_options* opts,
               void* stream) {
    if (!out) return ART_ERR_INVALID_ARG;
    *out = nullptr;
    if (nx <= 0 || ny <= 0 || nz <= 0) return ART_ERR_INVALID_ARG;
    const uint64_t N = (uint64_t)nx * ny * nz;
    if (N >= (1ull << 32)) return ART_ERR_INVALID_ARG;
    int rc = check_params(params);
    if (rc) return rc;
    art_options o;
    memset(&o, 0, sizeof o);
    if (opts) o = *opts;
    if (o.max_sources <= 0) return ART_ERR_INVALID_ARG;
    if (o.block_size == 0) o.block_size = 64;
    if (o.blocks_per_cu == 0) o.blocks_per_cu = 16;
    if (o.block_size < 64 || o.block_size > 256 || (o.block_size % 64) || o.blocks_per_cu < 1 ||
        o.blocks_per_cu > 64)
        return ART_ERR_INVALID_ARG;
    if (!(o.pool_mem_fraction > 0.0 && o.pool_mem_fraction <= 0.95)) o.pool_mem_fraction = 0.5;

    art_ctx* c = new (std::nothrow) art_ctx();
    if (!c) return ART_ERR_OUT_OF_MEMORY;
    c->nx = nx;
    c->ny = ny;
    c->nz = nz;
    c->N = N;
    c->p = *params;
    c->o = o;
    c->adj_block = o.block_size;
    c->adj_bpc = o.blocks_per_cu;
    c->stream = (hipStream_t)stream;
    if (hipGetDevice(&c->device) != hipSuccess ||
        hipDeviceGetAttribute(&c->cu_count, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess) {
        delete c;
        return ART_ERR_HIP;
    }
    init_geometry(c, nx, ny, nz, *params);
    // src, pix, tau (shared with the adjoint's G), tend; with the adjoint: child, last, rlast, taulast
    const uint64_t bytes_per_ray = 4 + 4 + 16 + 16 + (o.enable_adjoint ? 4 + 4 + 8 + 16 : 0);
    uint64_t cap = (uint64_t)o.pool_rays;
    if (cap == 0) {
        size_t free_b = 0, total_b = 0;
        if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
            delete c;
            return ART_ERR_HIP;
        }
        const uint64_t want = c->per_src_bound * (uint64_t)o.max_sources;
        const uint64_t fits = (uint64_t)((double)free_b * o.pool_mem_fraction) / bytes_per_ray;
        cap = std::min(want, fits);
    }
    cap = std::min<uint64_t>(cap, kMaxPoolRays);
    const uint64_t seeds = 12ull << (2 * params->level0);
    if (cap < seeds) {
        delete c;
        return ART_ERR_OUT_OF_MEMORY;
    }
    c->pool.cap = cap;
    uint64_t wave = cap / std::max<uint64_t>(c->per_src_bound, 1);
    if (wave < 1) wave = 1;  // a single source may still fit (the bound is loose)
    c->wave_max = (int)std::min<uint64_t>(wave, (uint64_t)o.max_sources);

    const bool det = params->deposit_mode == ART_DEPOSIT_DETERMINISTIC;
    const uint64_t ms = (uint64_t)o.max_sources;
    bool ok = dmalloc(&c->pool.src, cap) && dmalloc(&c->pool.pix, cap) && dmalloc(&c->pool.tau, 2 * cap) &&
              dmalloc(&c->pool.tend, 2 * cap) && dmalloc(&c->pool.tsum, (cap + kSplitTile - 1) / kSplitTile + 1) &&
              dmalloc(&c->ct, 1) && dmalloc(&c->st.created, ms * ART_MAX_LEVELS) &&
              dmalloc(&c->st.split, ms * ART_MAX_LEVELS) && dmalloc(&c->st.exited, ms * ART_MAX_LEVELS) &&
              dmalloc(&c->st.term, ms * ART_MAX_LEVELS) && dmalloc(&c->st.escaped, ms * 2) &&
              dmalloc(&c->st.residual, ms * 2) && dmalloc(&c->st.segments, ms) && dmalloc(&c->fscratch, 64) &&
              dmalloc(&c->ion, 4) && dmalloc(&c->rot, 9);
    if (ok && o.enable_adjoint)
        ok = dmalloc(&c->pool.child, cap) && dmalloc(&c->pool.last, cap) &&
             dmalloc(&c->pool.rlast, cap) && dmalloc(&c->pool.taulast, 2 * cap);
    c->pool.G = c->pool.tau;
    // one spare cell: the sweep's deposit cache flushes cells in pairs (2g, 2g + 1)
    if (ok) ok = det ? dmalloc(&c->det, 8 * (N + 1)) : dmalloc(&c->acc, 8 * (N + 1));
    if (ok) ok = dmalloc(&c->q, N) && dmalloc(&c->fg, N);
    if (ok) ok = dmalloc(&c->dirs, 3 * (uint64_t)kDirTable) && dmalloc(&c->sbound, ms) && dmalloc(&c->wtab, ms + 2);
    if (ok && o.enable_adjoint) ok = det ? dmalloc(&c->gdet, 2 * N) : dmalloc(&c->gk, 2 * N);
    if (ok && o.enable_adjoint) ok = dmalloc(&c->wv, N);
    if (ok) {
        c->ev.resize(2 * (ART_MAX_LEVELS + 1) * 64);
        for (auto& e : c->ev) ok = ok && hipEventCreate(&e) == hipSuccess;
        ok = ok && hipEventCreate(&c->ev_call0) == hipSuccess && hipEventCreate(&c->ev_call1) == hipSuccess;
    }
    if (!ok) {
        free_all(c);
        delete c;
        (void)hipGetLastError();
        return ART_ERR_OUT_OF_MEMORY;
    }
    if (hipMemcpy(c->rot, params->rot, 9 * sizeof(double), hipMemcpyHostToDevice) != hipSuccess) {
        free_all(c);
        delete c;
        return ART_ERR_HIP;
    }
    c->geo.rot = c->rot;
    hipLaunchKernelGGL(k_dir_table, dim3(64), dim3(256), 0, c->stream, c->dirs);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess) {
        free_all(c);
        delete c;
        return ART_ERR_HIP;
    }
    *out = c;
    return ART_OK;
}

int art_set_stream(art_ctx* c, void* stream) {
    if (!c) return ART_ERR_INVALID_ARG;
    c->stream = (hipStream_t)stream;
    return ART_OK;
}

namespace {

// The forward sweep on a context whose workspace is in place (art_trace's body,
// also run by art_trace_noalloc on its static workspace).
int trace_impl(art_ctx* c, const float* n_H, const float* x_n, const double* src_pos, const float* src_lum,
               int n_src, float* rate, float* force, float* J) {
    const bool det = c->p.deposit_mode == ART_DEPOSIT_DETERMINISTIC;
    const uint64_t N = c->N;
    const uint64_t ms = (uint64_t)c->o.max_sources;
    c->ev_used = 0;
    c->tape_ok = false;
    c->tape_gen = 0;
    if (c->timing) HIP_TRY(hipEventRecord(c->ev_call0, c->stream));
    int rc;
    if ((rc = begin_call(c, src_lum, n_src, n_H, x_n))) return rc;
    const int mode = J ? 2 : 1;
    const int lpe = mode == 2 ? 8 : 4;
    const uint64_t n_acc = N + (N & 1);  // whole pairs
    if (det) {
        if ((rc = zero(c, c->det, (uint64_t)lpe * n_acc))) return rc;
    } else if ((rc = zero(c, c->acc, (uint64_t)lpe * n_acc))) {
        return rc;
    }
    if ((rc = zero_stats(c, ms))) return rc;
    const SweepArgs a = sweep_args(c, n_H, x_n, src_pos, src_lum, force, J, n_src);
    int waves = 0;
    if ((rc = for_waves(c, src_pos, n_src, &waves, [&]() { return sweep_wave(c, a, mode); }))) return rc;
    const dim3 fg(fill_blocks(N)), fb(256);
    if (det)
        hipLaunchKernelGGL((k_finalize<true>), fg, fb, 0, c->stream, N, c->transparent, c->acc, c->det, lpe, c->ct,
                           rate, force, J, c->p.n_bins);
    else
        hipLaunchKernelGGL((k_finalize<false>), fg, fb, 0, c->stream, N, c->transparent, c->acc, c->det, lpe, c->ct,
                           rate, force, J, c->p.n_bins);
    HIP_TRY(hipGetLastError());
    if (c->timing) HIP_TRY(hipEventRecord(c->ev_call1, c->stream));
    c->last_nsrc = n_src;
    c->last_waves = waves;
    c->gen += 1;
    if (c->o.enable_adjoint && waves == 1) {
        c->tape_key[0] = n_H;
        c->tape_key[1] = x_n;
        c->tape_key[2] = src_pos;
        c->tape_key[3] = src_lum;
        c->tape_nsrc = n_src;
        c->tape_ok = true;
        c->tape_gen = c->gen;
    }
    return ART_OK;
}

}  // namespace

int art_trace(art_ctx* c, const float* n_H, const float* x_n, const double* src_pos, const float* src_lum,
              int n_src, float* rate, float* force, float* J) {
    if (!c || !n_H || !x_n || !rate || !force) return ART_ERR_INVALID_ARG;
    if (n_src < 0 || n_src > c->o.max_sources) return ART_ERR_INVALID_ARG;
    if (n_src > 0 && (!src_pos || !src_lum)) return ART_ERR_INVALID_ARG;
    return trace_impl(c, n_H, x_n, src_pos, src_lum, n_src, rate, force, J);
}

int art_get_tape(art_ctx* c, uint64_t* tape) {
    if (!c || !tape) return ART_ERR_INVALID_ARG;
    *tape = c->tape_ok ? c->tape_gen : 0;
    return ART_OK;
}

namespace {

// The adjoint's fixed-point scales (from the weights and the largest density),
// the cleared accumulator and the packed weights.  Then, after the levels'
// reverse sweeps, finalize.
int adjoint_prologue(art_ctx* c, const float* n_H, const float* src_lum, int n_src, const float* g_rate,
                     const float* g_force) {
    const bool det = c->p.deposit_mode == ART_DEPOSIT_DETERMINISTIC;
    const uint64_t N = c->N;
    int rc;
    if (det) {
        if ((rc = zero(c, (uint32_t*)c->fscratch, 2))) return rc;
        hipLaunchKernelGGL(k_adj_scale, dim3(fill_blocks(N) < 1024 ? fill_blocks(N) : 1024), dim3(256), 0,
                           c->stream, g_rate, g_force, n_H, N, c->fscratch);
        HIP_TRY(hipGetLastError());
        hipLaunchKernelGGL(k_adj_scale_final, dim3(1), dim3(64), 0, c->stream, c->ct, src_lum, n_src * c->p.n_bins,
                           c->fscratch, c->p.s_H, c->p.s_d);
        HIP_TRY(hipGetLastError());
        if ((rc = zero(c, c->gdet, 2 * N))) return rc;
    } else {
        if ((rc = zero(c, c->gk, 2 * N))) return rc;
    }
    hipLaunchKernelGGL(k_pack_wv, dim3(fill_blocks(N)), dim3(256), 0, c->stream, N, g_rate, g_force, c->wv);
    HIP_TRY(hipGetLastError());
    return ART_OK;
}

AdjArgs adjoint_args(art_ctx* c, const double* src_pos, const float* src_lum, int n_src) {
    AdjArgs aa;
    aa.g = c->geo;
    aa.q = c->q;
    aa.wv = c->wv;
    aa.src_pos = src_pos;
    aa.src_lum = src_lum;
    aa.pool = c->pool;
    aa.ct = c->ct;
    aa.gk = c->gk;
    aa.gdet = c->gdet;
    aa.N = (uint32_t)c->N;
    aa.n_src = (uint32_t)n_src;
    return aa;
}

int adjoint_levels(art_ctx* c, const AdjArgs& aa) {
    // the levels' claim counters start at zero for every walk over a tree
    hipLaunchKernelGGL(k_adj_reset, dim3(1), dim3(64), 0, c->stream, c->ct);
    HIP_TRY(hipGetLastError());
    for (int l = c->deepest; l >= c->p.level0; --l) {
        int rc = launch_adjoint(c, aa, l);
        if (rc) return rc;
    }
    return ART_OK;
}

int adjoint_epilogue(art_ctx* c, float* g_nH, float* g_xn) {
    const uint64_t N = c->N;
    const dim3 fg(fill_blocks(N)), fb(256);
    if (c->p.deposit_mode == ART_DEPOSIT_DETERMINISTIC)
        hipLaunchKernelGGL((k_adj_finalize<true>), fg, fb, 0, c->stream, N, c->gk, c->gdet, c->ct, c->transparent,
                           g_nH, g_xn);
    else
        hipLaunchKernelGGL((k_adj_finalize<false>), fg, fb, 0, c->stream, N, c->gk, c->gdet, c->ct, c->transparent,
                           g_nH, g_xn);
    HIP_TRY(hipGetLastError());
    return ART_OK;
}

int adjoint_check(art_ctx* c, const float* n_H, const float* x_n, const double* src_pos, const float* src_lum,
                  int n_src, const float* g_rate, const float* g_force, float* g_nH, float* g_xn) {
    if (!c || !n_H || !x_n || !g_rate || !g_force || !g_nH || !g_xn) return ART_ERR_INVALID_ARG;
    if (!c->o.enable_adjoint) return ART_ERR_NO_ADJOINT;
    if (n_src < 0 || n_src > c->o.max_sources) return ART_ERR_INVALID_ARG;
    if (n_src > 0 && (!src_pos || !src_lum)) return ART_ERR_INVALID_ARG;
    return ART_OK;
}

}  // namespace

int art_trace_adjoint(art_ctx* c, const float* n_H, const float* x_n, const double* src_pos, const float* src_lum,
                      int n_src, const float* g_rate, const float* g_force, float* g_nH, float* g_xn) {
    int rc = adjoint_check(c, n_H, x_n, src_pos, src_lum, n_src, g_rate, g_force, g_nH, g_xn);
    if (rc) return rc;
    // the pool is rebuilt here: no earlier tape survives
    c->tape_ok = false;
    c->tape_gen = 0;
    if ((rc = adjoint_prologue(c, n_H, src_lum, n_src, g_rate, g_force))) return rc;
    const AdjArgs aa = adjoint_args(c, src_pos, src_lum, n_src);
    // rebuild the tree wave by wave (tau recomputed, no segment storage), and walk
    // each wave's tree back before the next wave overwrites the pool
    if ((rc = begin_call(c, src_lum, n_src, n_H, x_n))) return rc;
    if ((rc = zero_stats(c, (uint64_t)c->o.max_sources))) return rc;
    const SweepArgs a = sweep_args(c, n_H, x_n, src_pos, src_lum, nullptr, nullptr, n_src);
    int waves = 0;
    rc = for_waves(c, src_pos, n_src, &waves, [&]() {
        int r = sweep_wave(c, a, 0);
        return r ? r : adjoint_levels(c, aa);
    });
    if (rc) return rc;
    c->last_nsrc = n_src;
    c->last_waves = waves;
    return adjoint_epilogue(c, g_nH, g_xn);
}

int art_trace_adjoint_tape(art_ctx* c, uint64_t tape, const float* n_H, const float* x_n, const double* src_pos,
                           const float* src_lum, int n_src, const float* g_rate, const float* g_force, float* g_nH,
                           float* g_xn) {
    int rc = adjoint_check(c, n_H, x_n, src_pos, src_lum, n_src, g_rate, g_force, g_nH, g_xn);
    if (rc) return rc;
    if (!(c->tape_ok && tape != 0 && tape == c->tape_gen && c->tape_key[0] == n_H && c->tape_key[1] == x_n &&
          c->tape_key[2] == src_pos && c->tape_key[3] == src_lum && c->tape_nsrc == n_src))
        return ART_ERR_NO_FORWARD;
    // the packed fields and the tree are the forward's (nothing has run since)
    if ((rc = adjoint_prologue(c, n_H, src_lum, n_src, g_rate, g_force))) return rc;
    if ((rc = adjoint_levels(c, adjoint_args(c, src_pos, src_lum, n_src)))) return rc;
    return adjoint_epilogue(c, g_nH, g_xn);
}

int art_trace_and_adjoint(art_ctx* c, const float* n_H, const float* x_n, const double* src_pos,
                          const float* src_lum, int n_src, float* rate, float* force, float* J,
                          const float* g_rate, const float* g_force, float* g_nH, float* g_xn) {
    int rc = adjoint_check(c, n_H, x_n, src_pos, src_lum, n_src, g_rate, g_force, g_nH, g_xn);
    if (rc) return rc;
    if (!rate || !force) return ART_ERR_INVALID_ARG;
    const bool det = c->p.deposit_mode == ART_DEPOSIT_DETERMINISTIC;
    const uint64_t N = c->N;
    c->ev_used = 0;
    c->tape_ok = false;
    c->tape_gen = 0;
    if (c->timing) HIP_TRY(hipEventRecord(c->ev_call0, c->stream));
    if ((rc = begin_call(c, src_lum, n_src, n_H, x_n))) return rc;
    const int mode = J ? 2 : 1;
    const int lpe = mode == 2 ? 8 : 4;
    const uint64_t n_acc = N + (N & 1);
    if (det) {
        if ((rc = zero(c, c->det, (uint64_t)lpe * n_acc))) return rc;
    } else if ((rc = zero(c, c->acc, (uint64_t)lpe * n_acc))) {
        return rc;
    }
    if ((rc = zero_stats(c, (uint64_t)c->o.max_sources))) return rc;
    if ((rc = adjoint_prologue(c, n_H, src_lum, n_src, g_rate, g_force))) return rc;
    const SweepArgs a = sweep_args(c, n_H, x_n, src_pos, src_lum, force, J, n_src);
    const AdjArgs aa = adjoint_args(c, src_pos, src_lum, n_src);
    // each wave's tree is walked back right after its forward sweep, while the
    // pool still holds it: no wave is traced twice
    int waves = 0;
    rc = for_waves(c, src_pos, n_src, &waves, [&]() {
        int r = sweep_wave(c, a, mode);
        return r ? r : adjoint_levels(c, aa);
    });
    if (rc) return rc;
    const dim3 fg(fill_blocks(N)), fb(256);
    if (det)
        hipLaunchKernelGGL((k_finalize<true>), fg, fb, 0, c->stream, N, c->transparent, c->acc, c->det, lpe, c->ct,
                           rate, force, J, c->p.n_bins);
    else
        hipLaunchKernelGGL((k_finalize<false>), fg, fb, 0, c->stream, N, c->transparent, c->acc, c->det, lpe, c->ct,
                           rate, force, J, c->p.n_bins);
    HIP_TRY(hipGetLastError());
    if ((rc = adjoint_epilogue(c, g_nH, g_xn))) return rc;
    if (c->timing) HIP_TRY(hipEventRecord(c->ev_call1, c->stream));
    c->last_nsrc = n_src;
    c->last_waves = waves;
    c->gen += 1;
    if (waves == 1) {  // the pool holds the whole tree: later adjoints may reuse it
        c->tape_key[0] = n_H;
        c->tape_key[1] = x_n;
        c->tape_key[2] = src_pos;
        c->tape_key[3] = src_lum;
        c->tape_nsrc = n_src;
        c->tape_ok = true;
        c->tape_gen = c->gen;
    }
    return ART_OK;
}

static int status_code(const Counters& h, uint64_t expected) {
    if (h.c.status & kStOverflow) return ART_ERR_QUEUE_OVERFLOW;
    if (h.c.status & kStOutside) return ART_ERR_SOURCE_OUTSIDE;
    if (h.c.status & kStBadField) return ART_ERR_BAD_FIELD;
    if (h.c.status & kStStuck) return ART_ERR_INVALID_ARG;
    if (h.c.destroy != expected) return ART_ERR_DESTROY_COUNT;
    return ART_OK;
}

static uint64_t destroy_expected(const art_ctx* c, int n_src) {
    return (uint64_t)n_src * (12ull << (2 * c->p.level_max));
}

int art_sync(art_ctx* c) {
    if (!c) return ART_ERR_INVALID_ARG;
    HIP_TRY(hipStreamSynchronize(c->stream));
    Counters h;
    HIP_TRY(hipMemcpy(&h, c->ct, sizeof h, hipMemcpyDeviceToHost));
    return status_code(h, destroy_expected(c, c->last_nsrc));
}

int art_get_stats(art_ctx* c, art_stats* out, int ns, uint32_t* created, uint32_t* split, uint32_t* exited,
                  uint32_t* terminated, double* escaped, double* residual, uint64_t* segments,
                  uint64_t* rays_bound) {
    if (!c || !out) return ART_ERR_INVALID_ARG;
    HIP_TRY(hipStreamSynchronize(c->stream));
    Counters h;
    HIP_TRY(hipMemcpy(&h, c->ct, sizeof h, hipMemcpyDeviceToHost));
    memset(out, 0, sizeof *out);
    out->n_src = c->last_nsrc;
    out->n_waves = (int)h.c.waves;
    out->segments = h.c.segments;
    out->destroy = h.c.destroy;
    out->destroy_expected = destroy_expected(c, c->last_nsrc);
    out->rays_max_wave = h.c.rays_wave_max;
    out->status = status_code(h, out->destroy_expected);
    const int n_all = c->last_nsrc;
    if (n_all > 0) {
        std::vector<uint32_t> buf((size_t)n_all * ART_MAX_LEVELS);
        uint32_t* dsrc[4] = {c->st.created, c->st.split, c->st.exited, c->st.term};
        uint32_t* hdst[4] = {created, split, exited, terminated};
        uint64_t* tot[4] = {out->created, out->split, out->exited, out->terminated};
        for (int k = 0; k < 4; ++k) {
            HIP_TRY(hipMemcpy(buf.data(), dsrc[k], buf.size() * 4, hipMemcpyDeviceToHost));
            for (int s = 0; s < n_all; ++s)
                for (int l = 0; l < ART_MAX_LEVELS; ++l) tot[k][l] += buf[(size_t)s * ART_MAX_LEVELS + l];
            if (hdst[k] && ns > 0)
                memcpy(hdst[k], buf.data(), (size_t)std::min(ns, n_all) * ART_MAX_LEVELS * 4);
        }
        const int m = std::min(ns, n_all);
        if (m > 0) {
            if (escaped) HIP_TRY(hipMemcpy(escaped, c->st.escaped, (size_t)m * 2 * 8, hipMemcpyDeviceToHost));
            if (residual) HIP_TRY(hipMemcpy(residual, c->st.residual, (size_t)m * 2 * 8, hipMemcpyDeviceToHost));
            if (segments) HIP_TRY(hipMemcpy(segments, c->st.segments, (size_t)m * 8, hipMemcpyDeviceToHost));
            if (rays_bound) {
                if (c->last_planned && c->sbound)
                    HIP_TRY(hipMemcpy(rays_bound, c->sbound, (size_t)m * 8, hipMemcpyDeviceToHost));
                else
                    memset(rays_bound, 0, (size_t)m * 8);
            }
        }
    }
    return ART_OK;
}

int art_set_timing(art_ctx* c, int enable) {
    if (!c) return ART_ERR_INVALID_ARG;
    c->timing = enable != 0;
    return ART_OK;
}

int art_get_timing(art_ctx* c, float* sweep_ms_total, int* sweep_launches, float* total_ms) {
    if (!c) return ART_ERR_INVALID_ARG;
    HIP_TRY(hipStreamSynchronize(c->stream));
    float tot = 0.0f;
    for (int i = 0; i + 1 < c->ev_used; i += 2) {
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, c->ev[i], c->ev[i + 1]));
        tot += ms;
    }
    if (sweep_ms_total) *sweep_ms_total = tot;
    if (sweep_launches) *sweep_launches = c->ev_used / 2;
    if (total_ms) {
        float ms = 0.0f;
        if (c->timing && hipEventElapsedTime(&ms, c->ev_call0, c->ev_call1) != hipSuccess) ms = 0.0f;
        *total_ms = ms;
    }
    return ART_OK;
}

}  // extern "C"

namespace {

// Launch shapes the autotuner tries: (threads per workgroup, workgroups per CU).
constexpr int kShapes[][2] = {{64, 8}, {64, 12}, {64, 16}, {128, 4}, {128, 6}, {256, 2}, {256, 4}};

// The best of `reps` timed runs after one untimed run (HIP events on the stream).
template <class F>
int best_time(art_ctx* c, int reps, F&& run, float* best) {
    *best = 1e30f;
    for (int rep = 0; rep <= reps; ++rep) {
        HIP_TRY(hipEventRecord(c->ev_call0, c->stream));
        int rc = run();
        if (rc) return rc;
        HIP_TRY(hipEventRecord(c->ev_call1, c->stream));
        HIP_TRY(hipEventSynchronize(c->ev_call1));
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, c->ev_call0, c->ev_call1));
        if (rep > 0) *best = std::min(*best, ms);
    }
    return ART_OK;
}

}  // namespace

extern "C" {

int art_autotune(art_ctx* c, const float* n_H, const float* x_n, const double* src_pos, const float* src_lum,
                 int n_src, float* rate, float* force, int* best_block, int* best_bpc, int* best_wave_sources,
                 float* best_ms) {
    if (!c || n_src < 1) return ART_ERR_INVALID_ARG;
    const art_options keep = c->o;
    const int keep_cap = c->wave_cap;
    const bool keep_timing = c->timing;
    c->timing = false;
    auto run = [&]() { return art_trace(c, n_H, x_n, src_pos, src_lum, n_src, rate, force, nullptr); };
    auto restore = [&](int rc) {
        c->o = keep;
        c->wave_cap = keep_cap;
        c->timing = keep_timing;
        return rc;
    };
    // 1. launch shapes, with as many sources per wave as the pool holds
    float best = 1e30f;
    int bb = keep.block_size, bp = keep.blocks_per_cu;
    c->wave_cap = 0;
    for (const auto& cd : kShapes) {
        c->o.block_size = cd[0];
        c->o.blocks_per_cu = cd[1];
        float ms;
        int rc = best_time(c, 2, run, &ms);
        if (rc) return restore(rc);
        if (ms < best) {
            best = ms;
            bb = cd[0];
            bp = cd[1];
        }
    }
    c->o.block_size = bb;
    c->o.blocks_per_cu = bp;
    // 2. sources per wave (fewer sources per wave: a smaller working set per level,
    //    but each wave repays the shallow levels and the launches)
    int bw = 0;
    const int full = std::min(wave_len(c), n_src);
    for (const int div : {2, 4}) {
        const int cap = (full + div - 1) / div;
        if (cap < 1 || cap >= full) continue;
        c->wave_cap = cap;
        float ms;
        int rc = best_time(c, 2, run, &ms);
        if (rc) return restore(rc);
        if (ms < best * 0.99f) {  // a clear gain only
            best = ms;
            bw = cap;
        }
    }
    c->wave_cap = bw;
    c->timing = keep_timing;
    if (best_block) *best_block = bb;
    if (best_bpc) *best_bpc = bp;
    if (best_wave_sources) *best_wave_sources = bw;
    if (best_ms) *best_ms = best;
    return art_sync(c);
}

int art_autotune_adjoint(art_ctx* c, const float* n_H, const float* x_n, const double* src_pos,
                         const float* src_lum, int n_src, float* rate, float* force, const float* g_rate,
                         const float* g_force, float* g_nH, float* g_xn, int* best_block, int* best_bpc,
                         float* best_ms) {
    if (!c || n_src < 1) return ART_ERR_INVALID_ARG;
    if (!c->o.enable_adjoint) return ART_ERR_NO_ADJOINT;
    const bool keep_timing = c->timing;
    c->timing = false;
    int rc = art_trace(c, n_H, x_n, src_pos, src_lum, n_src, rate, force, nullptr);
    c->timing = keep_timing;
    if (rc) return rc;
    c->timing = false;
    uint64_t tape = 0;
    art_get_tape(c, &tape);
    const int keep_b = c->adj_block, keep_p = c->adj_bpc;
    // over the stored tree when the sources fit one wave, else the full adjoint
    auto run = [&]() {
        return tape ? art_trace_adjoint_tape(c, tape, n_H, x_n, src_pos, src_lum, n_src, g_rate, g_force, g_nH, g_xn)
                    : art_trace_adjoint(c, n_H, x_n, src_pos, src_lum, n_src, g_rate, g_force, g_nH, g_xn);
    };
    float best = 1e30f;
    int bb = keep_b, bp = keep_p;
    for (const auto& cd : kShapes) {
        c->adj_block = cd[0];
        c->adj_bpc = cd[1];
        float ms;
        if ((rc = best_time(c, 2, run, &ms))) {
            c->adj_block = keep_b;
            c->adj_bpc = keep_p;
            c->timing = keep_timing;
            return rc;
        }
        if (ms < best) {
            best = ms;
            bb = cd[0];
            bp = cd[1];
        }
    }
    c->adj_block = bb;
    c->adj_bpc = bp;
    c->timing = keep_timing;
    if (best_block) *best_block = bb;
    if (best_bpc) *best_bpc = bp;
    if (best_ms) *best_ms = best;
    return art_sync(c);
}

int art_set_launch(art_ctx* c, int block_size, int blocks_per_cu) {
    if (!c) return ART_ERR_INVALID_ARG;
    if (block_size == 0) block_size = 64;
    if (blocks_per_cu == 0) blocks_per_cu = 16;
    if (block_size < 64 || block_size > 256 || (block_size % 64) || blocks_per_cu < 1 || blocks_per_cu > 64)
        return ART_ERR_INVALID_ARG;
    c->o.block_size = block_size;
    c->o.blocks_per_cu = blocks_per_cu;
    return ART_OK;
}

int art_set_adjoint_launch(art_ctx* c, int block_size, int blocks_per_cu) {
    if (!c) return ART_ERR_INVALID_ARG;
    if (block_size == 0) block_size = 64;
    if (blocks_per_cu == 0) blocks_per_cu = 16;
    if (block_size < 64 || block_size > 256 || (block_size % 64) || blocks_per_cu < 1 || blocks_per_cu > 64)
        return ART_ERR_INVALID_ARG;
    c->adj_block = block_size;
    c->adj_bpc = blocks_per_cu;
    return ART_OK;
}

int art_set_wave_sources(art_ctx* c, int max_sources_per_wave) {
    if (!c || max_sources_per_wave < 0) return ART_ERR_INVALID_ARG;
    c->wave_cap = max_sources_per_wave;
    c->tape_ok = false;
    c->tape_gen = 0;
    return ART_OK;
}

int art_set_transparent(art_ctx* c, const uint8_t* transparent) {
    if (!c) return ART_ERR_INVALID_ARG;
    c->transparent = transparent;
    c->tape_ok = false;
    return ART_OK;
}

int art_set_rotation(art_ctx* c, const double* rot) {
    if (!c || !rot) return ART_ERR_INVALID_ARG;
    Mat3 r;
    for (int i = 0; i < 9; ++i) {
        if (!std::isfinite(rot[i])) return ART_ERR_INVALID_ARG;
        r.m[i] = rot[i];
    }
    for (int i = 0; i < 3; ++i)  // rows orthonormal within 1e-6
        for (int j = 0; j < 3; ++j) {
            const double d = rot[3 * i] * rot[3 * j] + rot[3 * i + 1] * rot[3 * j + 1] + rot[3 * i + 2] * rot[3 * j + 2];
            if (fabs(d - (i == j ? 1.0 : 0.0)) > 1e-6) return ART_ERR_INVALID_ARG;
        }
    hipLaunchKernelGGL(k_set_rot, dim3(1), dim3(64), 0, c->stream, r, c->rot);
    HIP_TRY(hipGetLastError());
    c->tape_ok = false;
    return ART_OK;
}

int art_random_rotation(art_ctx* c, const double* u) {
    if (!c || !u) return ART_ERR_INVALID_ARG;
    hipLaunchKernelGGL(k_random_rot, dim3(1), dim3(64), 0, c->stream, u, c->rot);
    HIP_TRY(hipGetLastError());
    c->tape_ok = false;
    return ART_OK;
}

int art_get_rotation(art_ctx* c, double* rot) {
    if (!c || !rot) return ART_ERR_INVALID_ARG;
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(rot, c->rot, 9 * sizeof(double), hipMemcpyDeviceToHost));
    return ART_OK;
}

int art_ion_substep(art_ctx* c, const float* n_H, float* x_n, const double* src_pos, const float* src_lum,
                    int n_src, const art_ion_params* ip, double t_end, double* t_now, float* rate, float* force,
                    float* J, float* impulse) {
    if (!c || !ip || !t_now || !J) return ART_ERR_INVALID_ARG;
    if (!(ip->alpha_B >= 0.0) || !(ip->gamma_scale >= 0.0) || !(ip->C > 0.0) || std::isnan(t_end))
        return ART_ERR_INVALID_ARG;
    int rc = art_trace(c, n_H, x_n, src_pos, src_lum, n_src, rate, force, J);
    if (rc) return rc;
    const uint64_t N = c->N;
    const dim3 fg(fill_blocks(N)), fb(256);
    // the minimum: a few cells per thread and one atomic per block at most
    const dim3 mg(std::min(fill_blocks(N), 1024));
    hipLaunchKernelGGL(k_ion_begin, dim3(1), dim3(64), 0, c->stream, c->ion);
    hipLaunchKernelGGL(k_ion_minq, mg, fb, 0, c->stream, N, n_H, (const float*)x_n, (const float*)J, c->transparent,
                       ip->gamma_scale, ip->alpha_B, c->ion);
    hipLaunchKernelGGL(k_ion_dt, dim3(1), dim3(64), 0, c->stream, c->ion, ip->C, t_end, t_now);
    hipLaunchKernelGGL(k_ion_update, fg, fb, 0, c->stream, N, n_H, x_n, (const float*)J, (const float*)force,
                       (const uint8_t*)c->transparent, impulse, ip->gamma_scale, ip->alpha_B,
                       (const unsigned long long*)c->ion);
    HIP_TRY(hipGetLastError());
    // x_n changed in place: the tree just traced no longer belongs to the inputs
    c->tape_ok = false;
    c->tape_gen = 0;
    return ART_OK;
}

int art_ion_subcycle(art_ctx* c, const float* n_H, float* x_n, const double* src_pos, const float* src_lum,
                     int n_src, const art_ion_params* ip, double t_end, int max_substeps, float* rate,
                     float* force, float* J, float* impulse, int* n_substeps, double* t_reached) {
    if (!c || !ip || max_substeps < 0 || std::isnan(t_end)) return ART_ERR_INVALID_ARG;
    double* clock = (double*)(c->ion + 2);
    hipLaunchKernelGGL(k_fill_f64, dim3(1), dim3(64), 0, c->stream, clock, (uint64_t)1);
    HIP_TRY(hipGetLastError());
    double t = 0.0;
    int k = 0;
    int rc = ART_OK;
    while (k < max_substeps && t < t_end) {
        if ((rc = art_ion_substep(c, n_H, x_n, src_pos, src_lum, n_src, ip, t_end, clock, rate, force, J, impulse)))
            break;
        ++k;
        if ((rc = art_sync(c))) break;
        HIP_TRY(hipMemcpy(&t, clock, sizeof(double), hipMemcpyDeviceToHost));
    }
    if (n_substeps) *n_substeps = k;
    if (t_reached) *t_reached = t;
    return rc;
}

void art_destroy(art_ctx* c) {
    if (!c) return;
    (void)hipStreamSynchronize(c->stream);
    free_all(c);
    delete c;
}

}  // extern "C"

// --------------------------------------------------------------------------
// Forward sweep without any allocation (art_trace_noalloc)
// --------------------------------------------------------------------------

// The workspace of art_trace_noalloc: one array per GPU, held until the process
// ends.  In host code `scratch` names a host-side stand-in, not the device
// array: kernels and copies get the address hipGetSymbolAddress returns for the
// current device.
constexpr size_t kScratchBytes = (size_t)ART_NOALLOC_SCRATCH_MIB << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch[kMaxDevices];

// The device address of `scratch` on the current device, looked up once per device.
int scratch_on_device(int dev, unsigned char** out) {
    if (dev < 0 || dev >= kMaxDevices) return ART_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void* p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return ART_ERR_HIP;
        g_scratch[dev] = (unsigned char*)p;
    }
    *out = g_scratch[dev];
    return ART_OK;
}

// Carves the workspace of one call out of [base, base + kScratchBytes): counters,
// per-source statistics, the rotation, the packed fields, the accumulator and,
// in what is left, the ray pool.  Returns false if the fixed parts or the seeds
// of one source do not fit.
struct Carver {
    unsigned char* base;
    size_t used = 0;
    template <class T>
    T* take(uint64_t n) {
        used = (used + 255) & ~(size_t)255;
        T* p = (T*)(base + used);
        used += (size_t)n * sizeof(T);
        return p;
    }
};

bool noalloc_layout(art_ctx* c, unsigned char* base, int n_src, bool want_J) {
    Carver cv{base};
    const uint64_t N = c->N;
    const uint64_t ms = (uint64_t)std::max(1, n_src);
    c->ct = cv.take<Counters>(1);
    c->st.created = cv.take<uint32_t>(ms * ART_MAX_LEVELS);
    c->st.split = cv.take<uint32_t>(ms * ART_MAX_LEVELS);
    c->st.exited = cv.take<uint32_t>(ms * ART_MAX_LEVELS);
    c->st.term = cv.take<uint32_t>(ms * ART_MAX_LEVELS);
    c->st.escaped = cv.take<double>(ms * 2);
    c->st.residual = cv.take<double>(ms * 2);
    c->st.segments = cv.take<unsigned long long>(ms);
    c->rot = cv.take<double>(9);
    c->q = cv.take<float2>(N);
    c->fg = cv.take<float>(N);
    const uint64_t n_acc = (uint64_t)(want_J ? 8 : 4) * (N + (N & 1));
    if (c->p.deposit_mode == ART_DEPOSIT_DETERMINISTIC) c->det = cv.take<unsigned long long>(n_acc);
    else c->acc = cv.take<float>(n_acc);
    if (cv.used + 4096 > kScratchBytes) return false;
    // the pool: 40 bytes per ray plus a tile count per kSplitTile rays, and padding
    const uint64_t room = kScratchBytes - cv.used - 5 * 256;
    uint64_t cap = (room - 8) / (40 + 1);
    cap = std::min<uint64_t>(cap, kMaxPoolRays);
    c->pool.tsum = cv.take<uint32_t>((cap + kSplitTile - 1) / kSplitTile + 1);
    c->pool.tau = cv.take<double>(2 * cap);
    c->pool.tend = cv.take<double>(2 * cap);
    c->pool.src = cv.take<uint32_t>(cap);
    c->pool.pix = cv.take<uint32_t>(cap);
    if (cv.used > kScratchBytes) return false;
    c->pool.cap = cap;
    return cap >= (12ull << (2 * c->p.level0));
}

// The status art_sync would report, written to the caller's device int.
__global__ void k_status_out(const Counters* ct, unsigned long long expected, int* out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    const uint32_t s = ct->c.status;
    int rc = ART_OK;
    if (s & kStOverflow) rc = ART_ERR_QUEUE_OVERFLOW;
    else if (s & kStOutside) rc = ART_ERR_SOURCE_OUTSIDE;
    else if (s & kStBadField) rc = ART_ERR_BAD_FIELD;
    else if (s & kStStuck) rc = ART_ERR_INVALID_ARG;
    else if (ct->c.destroy != expected) rc = ART_ERR_DESTROY_COUNT;
    *out = rc;
}

}  // namespace

extern "C" int art_trace_noalloc(int nx, int ny, int nz, const art_params* params, const float* n_H,
                                 const float* x_n, const double* src_pos, const float* src_lum, int n_src,
                                 float* rate, float* force, float* J, int* status, void* stream) {
    if (nx <= 0 || ny <= 0 || nz <= 0 || !n_H || !x_n || !rate || !force || n_src < 0) return ART_ERR_INVALID_ARG;
    if (n_src > 0 && (!src_pos || !src_lum)) return ART_ERR_INVALID_ARG;
    int rc = check_params(params);
    if (rc) return rc;
    const uint64_t N = (uint64_t)nx * ny * nz;
    if (N >= (1ull << 32)) return ART_ERR_INVALID_ARG;
    art_ctx c{};
    c.nx = nx;
    c.ny = ny;
    c.nz = nz;
    c.N = N;
    c.p = *params;
    c.o.max_sources = std::max(1, n_src);
    c.o.block_size = 64;
    c.o.blocks_per_cu = 16;
    c.stream = (hipStream_t)stream;
    init_geometry(&c, nx, ny, nz, *params);
    // sizes first, on a null base: no device is touched for an input that cannot fit
    if (!noalloc_layout(&c, nullptr, n_src, J != nullptr)) return ART_ERR_TOO_LARGE;
    if (hipGetDevice(&c.device) != hipSuccess ||
        hipDeviceGetAttribute(&c.cu_count, hipDeviceAttributeMultiprocessorCount, c.device) != hipSuccess)
        return ART_ERR_HIP;
    unsigned char* base = nullptr;
    if ((rc = scratch_on_device(c.device, &base))) return rc;
    noalloc_layout(&c, base, n_src, J != nullptr);
    c.wave_max = (int)std::max<uint64_t>(1, std::min<uint64_t>(c.pool.cap / std::max<uint64_t>(c.per_src_bound, 1),
                                                                (uint64_t)c.o.max_sources));
    Mat3 r;
    for (int i = 0; i < 9; ++i) r.m[i] = params->rot[i];
    hipLaunchKernelGGL(k_set_rot, dim3(1), dim3(64), 0, c.stream, r, c.rot);
    HIP_TRY(hipGetLastError());
    c.geo.rot = c.rot;
    if ((rc = trace_impl(&c, n_H, x_n, src_pos, src_lum, n_src, rate, force, J))) return rc;
    if (status) {
        hipLaunchKernelGGL(k_status_out, dim3(1), dim3(64), 0, c.stream, c.ct,
                           (unsigned long long)destroy_expected(&c, n_src), status);
        HIP_TRY(hipGetLastError());
    }
    return ART_OK;
}
