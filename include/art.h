/*
 * art.h -- C ABI of the MI355X (gfx950) adaptive ray tracing (ART) sweep.
 *
 * The sweep follows Kim, Kim, Ostriker & Skinner (2017), Sec. 2.1 "Adaptive Ray
 * Tracing": photon packets leave each point source along HEALPix directions
 * (N_ray(l) = 12*4^l equal-area pixels, packet luminosity L/N_ray(l0)), are
 * marched cell by cell through a uniform Cartesian grid, lose
 * Delta L = L_in (1 - e^{-Delta tau}) with Delta tau = chi Delta r in every cell
 * they cross, deposit that luminosity and the momentum n Delta L / c there
 * (Eqs. e:RT2, e:Erad, e:Frad), split into the four HEALPix children at
 * r_max(l) = sqrt(3/(pi m_ray)) 2^l dx, and end at the domain boundary or once
 * the optical depth from the source exceeds tau_term in every frequency bin.
 * The opacities are those of Sec. 2.3: chi_i = n_H (x_n sigma_H + sigma_d) for
 * the ionizing bin, chi_n = n_H sigma_d for the non-ionizing bin.
 *
 * Units and coordinates: lengths are in cells (dx = 1), measured from the
 * domain's lower corner, which is the origin: the domain is
 * [0,nx) x [0,ny) x [0,nz), cell (i, j, k) occupies [i,i+1) x [j,j+1) x [k,k+1),
 * and source positions are given in these coordinates.  A caller with a
 * physical cell size dx and origin x0 passes (x - x0) / dx and folds dx into the
 * opacities: s_H = sigma_H dx and s_d = sigma_d dx are optical depths per cell
 * length per unit density.  Cell volume 1, c = 1, h nu_i = 1.
 * Field layout: a flat array of nx*ny*nz values with x fastest: index
 * (k*ny + j)*nx + i.
 * Frequency bins: bin 0 is ionizing (gas and dust opacity), bin 1 (if n_bins
 * is 2) non-ionizing (dust only).
 *
 * Memory ownership: every pointer argument of art_trace / art_trace_adjoint is
 * DEVICE memory owned by the caller.  The library owns only its workspace (ray
 * pool, counters, accumulators), allocated in art_create and freed in
 * art_destroy.  Outputs are overwritten, never accumulated.
 *
 * Streams: art_trace and art_trace_adjoint only enqueue kernels on the
 * context's stream (no host synchronisation, no allocation, no memset nodes),
 * so they can be captured into a HIP graph.  Device-side failures (ray pool
 * overflow, a source outside the domain, a broken destroy count) are recorded
 * in a device status word and reported by art_sync / art_get_stats, which
 * synchronise the stream.
 *
 * Errors: every function returns ART_OK (0) or a negative ART_ERR_* code; no
 * exception or abort crosses the ABI.  art_strerror names a code.
 */
#ifndef ART_H
#define ART_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ART_OK 0
#define ART_ERR_INVALID_ARG (-1)      /* bad size, level, pointer or parameter */
#define ART_ERR_HIP (-2)              /* a HIP runtime call failed */
#define ART_ERR_OUT_OF_MEMORY (-3)    /* workspace allocation failed in art_create */
#define ART_ERR_QUEUE_OVERFLOW (-4)   /* device: the ray pool filled up (no ray is dropped silently) */
#define ART_ERR_SOURCE_OUTSIDE (-5)   /* device: a source position lies outside the domain */
#define ART_ERR_DESTROY_COUNT (-6)    /* device: ended rays do not add up to N_src*12*4^level_max */
#define ART_ERR_NO_FORWARD (-7)       /* art_trace_adjoint_tape: no stored forward tree matches the call */
#define ART_ERR_BAD_FIELD (-8)        /* device: a cell has n_H < 0 or not finite, or x_n outside [0, 1] */
#define ART_ERR_NO_ADJOINT (-9)       /* adjoint requested on a context built without adjoint support */
#define ART_ERR_TOO_LARGE (-10)       /* art_trace_noalloc: the input does not fit its static workspace */

#define ART_DEPOSIT_ATOMIC 0          /* FP32 hardware atomics (fast, order-dependent rounding) */
#define ART_DEPOSIT_DETERMINISTIC 1   /* 64-bit fixed-point integer sums: bitwise reproducible */

#define ART_MAX_LEVELS 16
#define ART_MAX_BINS 2

/* Method parameters (Sec. 2.1, Sec. 2.3). */
typedef struct {
    int level0;          /* initial HEALPix level l0 (12*4^l0 rays per source) */
    int level_max;       /* deepest level; rays at level_max never split; < ART_MAX_LEVELS */
    double phi_c;        /* m_ray: split when (dx/r)^2 < m_ray * Omega_ray */
    double tau_term;     /* destroy a ray once tau_b > tau_term in every bin; 0 < tau_term < 5e5 */
    double s_H;          /* sigma_H * dx in code units: ionizing gas opacity per unit n_H x_n */
    double s_d;          /* sigma_d * dx in code units: dust opacity per unit n_H */
    int n_bins;          /* 1 (ionizing only) or 2 (ionizing, non-ionizing) */
    double rot[9];       /* row-major rotation applied to every HEALPix direction */
    int deposit_mode;    /* ART_DEPOSIT_ATOMIC or ART_DEPOSIT_DETERMINISTIC */
} art_params;

/* Workspace and launch options fixed at art_create. */
typedef struct {
    int max_sources;         /* largest n_src accepted by art_trace */
    int enable_adjoint;      /* 1: also allocate the adjoint workspace */
    int64_t pool_rays;       /* ray-pool capacity (rays per source wave, at most 2^32 - 2^23;
                                larger values are reduced to that); 0 = size automatically */
    double pool_mem_fraction;/* automatic sizing: at most this fraction of free HBM (0 -> 0.5) */
    int block_size;          /* threads per workgroup of the sweep kernels (64, 128, 192 or 256; 0 -> 64) */
    int blocks_per_cu;       /* workgroups per CU launched for each sweep (0 -> 16) */
} art_options;

/* Per-trace statistics (host copy).  Per-source arrays are indexed [src][level]
 * or [src][bin] and hold the first min(n_src, stats_sources) sources. */
typedef struct {
    int status;                    /* ART_OK or the first device-side error of the last call */
    int n_src;                     /* sources in the last art_trace */
    int n_waves;                   /* source waves of the last call that traced at least one source */
    uint64_t segments;             /* ray-cell segments deposited (all sources) */
    uint64_t destroy;              /* sum over ended rays of 4^(level_max - level) */
    uint64_t destroy_expected;     /* n_src * 12 * 4^level_max */
    uint64_t rays_max_wave;        /* largest number of rays held by one source wave */
    uint64_t created[ART_MAX_LEVELS], split[ART_MAX_LEVELS];
    uint64_t exited[ART_MAX_LEVELS], terminated[ART_MAX_LEVELS];
} art_stats;

typedef struct art_ctx art_ctx;

/* Create a context for an nx*ny*nz grid.  `stream` is a hipStream_t (NULL = the
 * null stream).  Allocates the workspace; returns ART_ERR_OUT_OF_MEMORY if it
 * does not fit.  On success *ctx is owned by the caller until art_destroy. */
int art_create(art_ctx **ctx, int nx, int ny, int nz, const art_params *params,
               const art_options *opts, void *stream);

/* Change the stream later calls are enqueued on. */
int art_set_stream(art_ctx *ctx, void *stream);

/* Forward ART sweep (Sec. 2.1).
 *   n_H     [N]        total hydrogen density per cell (float, >= 0)
 *   x_n     [N]        neutral fraction per cell (float, in [0, 1])
 *   src_pos [n_src][3] source positions in cell units (double), inside [0,nx)x[0,ny)x[0,nz)
 *   src_lum [n_src][n_bins] source luminosity per bin (float, >= 0)
 *   rate    [N]        out: photoionizations per unit time (Eq. e:photrate2): the
 *                      gas's share x_n s_H / (x_n s_H + s_d) of the ionizing
 *                      luminosity absorbed in the cell, i.e. s_H x_n n_H J_0
 *   force   [3][N]     out: absorbed momentum per unit time, sum over bins of
 *                      Delta L n (chi F / c, Eq. e:radforce), structure of arrays
 *   J       [n_bins][N] out (may be NULL): sum of L_in dr (1-e^{-dtau})/dtau per cell,
 *                      i.e. c E dV of Eq. e:Erad with the chi -> 0 limit taken
 * All sources share one ray pool; they are traced together in waves of as many
 * sources as the pool holds: if a geometric bound shared by every source needs
 * more than one wave, the device plans the waves from a bound on each source's
 * own rays (no host synchronisation).  Asynchronous on the context's stream.
 * On a context with adjoint support, a trace done in one wave keeps its ray tree
 * in the pool as a tape for art_trace_adjoint_tape (see art_get_tape). */
int art_trace(art_ctx *ctx, const float *n_H, const float *x_n, const double *src_pos,
              const float *src_lum, int n_src, float *rate, float *force, float *J);

/* Token of the tape the last art_trace left (nonzero), or 0 if there is none: the
 * context has no adjoint support, the trace needed several source waves, or a
 * later call overwrote the pool or changed what the tree depends on
 * (art_trace_adjoint, art_ion_substep, art_set_transparent, art_set_rotation,
 * art_random_rotation, another art_trace).  Host-side only. */
int art_get_tape(art_ctx *ctx, uint64_t *tape);

/* Reverse-mode derivative of loss = sum_c g_rate[c] rate[c] + sum_c g_force[.][c] . force[.][c]
 * with respect to n_H and x_n, holding the ray tree of the forward sweep fixed
 * (the same splits, exits and optical-depth terminations; Sec. 2.1 splitting is
 * geometric, so the tree changes only where a termination flips).
 *   g_rate [N], g_force [3][N]  in (device, float)
 *   g_nH [N], g_xn [N]          out (device, float), overwritten
 * n_H, x_n and the sources are those of the forward sweep to differentiate.
 * Requires enable_adjoint (else ART_ERR_NO_ADJOINT).  Rebuilds the ray tree
 * from these inputs, wave by wave (every segment's optical depth is recomputed,
 * no segment is stored), so it needs no preceding art_trace and overwrites any
 * stored tape. */
int art_trace_adjoint(art_ctx *ctx, const float *n_H, const float *x_n, const double *src_pos,
                      const float *src_lum, int n_src, const float *g_rate,
                      const float *g_force, float *g_nH, float *g_xn);

/* The same derivative over the tree a preceding art_trace stored, without
 * tracing it again.  tape is the token art_get_tape returned after that trace,
 * and n_H, x_n, src_pos, src_lum, n_src are the same pointers and count that
 * trace was given; their contents must not have changed since (the library
 * cannot check contents).  The tape stays valid, so several adjoints (other
 * g_rate, g_force) may follow one trace.  ART_ERR_NO_FORWARD, with nothing
 * enqueued, if the token is not that of the context's valid tape or the
 * pointers differ from the trace's; otherwise as art_trace_adjoint. */
int art_trace_adjoint_tape(art_ctx *ctx, uint64_t tape, const float *n_H, const float *x_n,
                           const double *src_pos, const float *src_lum, int n_src,
                           const float *g_rate, const float *g_force, float *g_nH, float *g_xn);

/* art_trace and the adjoint of loss = <g_rate, rate> + <g_force, force> in one
 * call, for callers that know the loss's weights when they trace (a loss that is
 * linear in the outputs, or its linearisation at known weights).  Each source
 * wave's tree is walked back right after that wave's forward sweep, so no tree
 * is traced twice however many waves the sources need.  Arguments as art_trace
 * and art_trace_adjoint (J may be NULL); requires enable_adjoint.  Leaves a tape
 * (art_get_tape) when the sources fit one wave. */
int art_trace_and_adjoint(art_ctx *ctx, const float *n_H, const float *x_n, const double *src_pos,
                          const float *src_lum, int n_src, float *rate, float *force, float *J,
                          const float *g_rate, const float *g_force, float *g_nH, float *g_xn);

/* Synchronise the stream and return the device status of the last call. */
int art_sync(art_ctx *ctx);

/* Synchronise and copy the statistics of the last art_trace (and per-source
 * arrays, each [stats_sources][ART_MAX_LEVELS], [stats_sources][ART_MAX_BINS] or
 * [stats_sources], any of which may be NULL).  src_rays_bound: the bound on each
 * source's rays that planned the source waves on the device (all zero if the last
 * call did not plan them there: one wave, or a tuned cap on sources per wave). */
int art_get_stats(art_ctx *ctx, art_stats *out, int stats_sources, uint32_t *src_created,
                  uint32_t *src_split, uint32_t *src_exited, uint32_t *src_terminated,
                  double *src_escaped, double *src_residual, uint64_t *src_segments,
                  uint64_t *src_rays_bound);

/* Autotuning (times real runs on the given inputs, synchronises; outputs hold the
 * last run).  art_autotune times the forward sweep for each launch shape of a
 * built-in list (threads per workgroup x workgroups per CU), then, with the
 * fastest shape, caps of n_src/2 and n_src/4 sources per wave against as many as
 * the pool holds (a cap is kept only if at least 1% faster); it keeps the winners
 * in the context and writes them (best_wave_sources 0 = no cap) with the best time
 * in milliseconds.  Any output pointer may be NULL. */
int art_autotune(art_ctx *ctx, const float *n_H, const float *x_n, const double *src_pos,
                 const float *src_lum, int n_src, float *rate, float *force,
                 int *best_block_size, int *best_blocks_per_cu, int *best_wave_sources, float *best_ms);

/* The same for the adjoint sweep's launch shape (separate from the forward's): one
 * art_trace, then adjoints over its stored tree (or full adjoints if the sources
 * need several waves) for each shape.  Requires enable_adjoint. */
int art_autotune_adjoint(art_ctx *ctx, const float *n_H, const float *x_n, const double *src_pos,
                         const float *src_lum, int n_src, float *rate, float *force,
                         const float *g_rate, const float *g_force, float *g_nH, float *g_xn,
                         int *best_block_size, int *best_blocks_per_cu, float *best_ms);

/* Set the launch shape of the sweep kernels (as art_options.block_size and
 * blocks_per_cu; 0 selects the default), e.g. a shape art_autotune found earlier
 * for the same grid and source count.  ART_ERR_INVALID_ARG for a shape outside the
 * ranges art_create accepts. */
int art_set_launch(art_ctx *ctx, int block_size, int blocks_per_cu);

/* The same for the adjoint sweep kernels (art_create starts them at the forward's). */
int art_set_adjoint_launch(art_ctx *ctx, int block_size, int blocks_per_cu);

/* Trace at most this many sources per wave (0: as many as the pool holds).  Results
 * do not depend on it (bitwise, in the deterministic mode); with more than one wave
 * no tape is kept.  Clears the stored tape. */
int art_set_wave_sources(art_ctx *ctx, int max_sources_per_wave);

/* Average duration in ms of the per-level sweep launches of the last forward
 * call (HIP events on the context's stream; enable with art_set_timing). */
int art_set_timing(art_ctx *ctx, int enable);
int art_get_timing(art_ctx *ctx, float *sweep_ms_total, int *sweep_launches, float *total_ms);

/* ---- Sink control volumes (Sec. 4.1) -------------------------------------------
 *
 * The gas in a star particle's control volume is invisible to the radiation: such
 * cells are transparent.  transparent is a device array of N bytes owned by the caller (nonzero =
 * such a cell), or NULL for none; it stays in use until replaced, so it must stay
 * valid for every later call.  In flagged cells the gas neither absorbs nor receives
 * photons: no opacity, no rate, no force (J still holds the radiation passing
 * through), zero gradients from art_trace_adjoint, and art_ion_substep leaves x_n
 * unchanged and takes no substep limit from them.  Host-side only (no launch). */
int art_set_transparent(art_ctx *ctx, const uint8_t *transparent);

/* ---- Rotation of the ray directions (Sec. 2.1) --------------------------------
 *
 * Every HEALPix direction is multiplied by a rotation before it is traced; the
 * paper rotates the injection directions at random every time step to smear the
 * geometric artefacts of the crossing-length deposit.  The rotation lives in
 * device memory: it starts as art_params.rot and applies to every later
 * art_trace / art_trace_adjoint / art_ion_substep on the context (an adjoint whose
 * forward tree was traced under another rotation retraces the tree). */

/* Set the rotation (host array of 9 doubles, row-major; rows orthonormal within
 * 1e-6, else ART_ERR_INVALID_ARG).  Asynchronous on the context's stream. */
int art_set_rotation(art_ctx *ctx, const double *rot);

/* Set a uniformly distributed (Haar) random rotation drawn from u, a device
 * pointer to three numbers in [0, 1) supplied by the caller: the unit quaternion
 * (sqrt(1-u0) sin 2 pi u1, sqrt(1-u0) cos 2 pi u1, sqrt(u0) sin 2 pi u2,
 * sqrt(u0) cos 2 pi u2) of Shoemake's construction.  Asynchronous and
 * graph-capturable: a captured call reads u when the graph runs. */
int art_random_rotation(art_ctx *ctx, const double *u);

/* Synchronise the stream and copy the current rotation to rot (host, 9 doubles). */
int art_get_rotation(art_ctx *ctx, double *rot);

/* ---- Ionization subcycle around the sweep (Sec. 2.3) -------------------------
 *
 * The source update of the neutral fraction, dx_n/dt = alpha_B n_e (1 - x_n) -
 * x_n Gamma with n_e = n_H (1 - x_n) (Eq. e:xn), advanced in substeps between
 * sweeps.  Units are the caller's, as long as they are consistent: alpha_B n_H is
 * a rate per unit time, and Gamma = gamma_scale J_0 is the photoionization rate
 * per neutral atom, where J_0 is the sweep's ionizing-bin J (so gamma_scale =
 * s_H / V_cell, the cross-section per cell length over the cell volume). */
typedef struct {
    double alpha_B;      /* case-B recombination coefficient (>= 0) */
    double gamma_scale;  /* Gamma = gamma_scale * J_0 (>= 0) */
    double C;            /* substep coefficient of Eq. e:dtss (> 0; the paper uses 0.1) */
} art_ion_params;

/* One radiation substep (Sec. 2.3, the subcycle after the hydro update):
 *   1. art_trace of the current x_n (rate, force and J are written as art_trace
 *      writes them; J must hold n_bins*N floats, bin 0 being the ionizing one);
 *   2. dt = min(C * min over cells with n_H > 0 of n_H / |I - R|, t_end - *t_now)
 *      (Eq. e:dtss), with I = Gamma n_H x_n and R = alpha_B n_e^2; dt = 0 once
 *      *t_now >= t_end;
 *   3. x_n <- x_eq0 + (x_n - x_eq0) exp(-dt (Gamma + alpha_B n_e)), x_eq0 =
 *      alpha_B n_e / (Gamma + alpha_B n_e), n_e from the substep's start (Method B,
 *      Eq. e:xn3), in FP64 per cell, stored as float32 in place;
 *   4. impulse[3][N] += force * dt if impulse is not NULL (the momentum kick of the
 *      radiation force over the substep, in the force's units times time);
 *   5. *t_now += dt (set to t_end exactly when the substep reaches it).
 * t_now is a device pointer to one double.  Everything is asynchronous on the
 * context's stream and capturable in a HIP graph (no host synchronisation, no
 * allocation); the device status is reported by art_sync.  The dt taken can be
 * read back from *t_now.  Errors: ART_ERR_INVALID_ARG for a NULL argument, a
 * negative alpha_B or gamma_scale, or C <= 0; the errors of art_trace. */
int art_ion_substep(art_ctx *ctx, const float *n_H, float *x_n, const double *src_pos,
                    const float *src_lum, int n_src, const art_ion_params *ip, double t_end,
                    double *t_now, float *rate, float *force, float *J, float *impulse);

/* The subcycle of one hydro step: substeps from t = 0 until t_end (or until
 * max_substeps have run), synchronising after each to read the time reached and
 * the device status.  Writes the number of substeps and the time reached (either
 * pointer may be NULL).  x_n, rate, force, J and impulse as in art_ion_substep;
 * impulse (if not NULL) accumulates over the whole subcycle. */
int art_ion_subcycle(art_ctx *ctx, const float *n_H, float *x_n, const double *src_pos,
                     const float *src_lum, int n_src, const art_ion_params *ip, double t_end,
                     int max_substeps, float *rate, float *force, float *J, float *impulse,
                     int *n_substeps, double *t_reached);

void art_destroy(art_ctx *ctx);
const char *art_strerror(int code);

/* ---- Forward sweep for callers that cannot allocate ------------------------------
 *
 * For code that may not call hipMalloc or create a context: under HIP graph
 * capture, in tight serving loops, or in harnesses that forbid allocation.  The same
 * forward sweep as art_trace (same kernels, same results: bitwise in the
 * deterministic mode), with no context: the workspace (counters, per-source
 * statistics, packed fields, accumulator, ray pool) lives in a static device array
 * of ART_NOALLOC_SCRATCH_MIB MiB that the library holds on every GPU it runs on
 * until the process ends.  Nothing is allocated or freed, by the library or by a
 * library it calls.
 *   nx, ny, nz, params       grid and method parameters as for art_create
 *   n_H .. J                 as for art_trace (device memory owned by the caller)
 *   status                   device int (may be NULL): after the call completes on
 *                            the stream it holds ART_OK or the device-side error
 *                            art_sync would report
 *   stream                   hipStream_t the kernels are enqueued on (NULL = null stream)
 * Sources are traced in waves that fit what is left of the array after the
 * fixed parts (about 76 bytes per cell and 300 per source), at 40 bytes per ray.
 * ART_ERR_TOO_LARGE, with nothing enqueued, if the fixed parts or one source's
 * seed rays do not fit; a tree larger than the pool is reported as
 * ART_ERR_QUEUE_OVERFLOW in *status.  Every call on a GPU uses that GPU's one
 * array (it keeps the last call's contents; the call clears what it needs), so
 * calls that overlap on one GPU, on different streams or threads, race. */
#define ART_NOALLOC_SCRATCH_MIB 64
int art_trace_noalloc(int nx, int ny, int nz, const art_params *params, const float *n_H,
                      const float *x_n, const double *src_pos, const float *src_lum, int n_src,
                      float *rate, float *force, float *J, int *status, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* ART_H */
