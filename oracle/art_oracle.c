/*
 * art_oracle.c -- plain, slow FP64 CPU oracle of the adaptive ray tracing (ART)
 * sweep of Kim, Kim, Ostriker & Skinner (2017), Sec. 2.1 "Adaptive Ray Tracing".
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or load
 * this file: only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark use it.  It shares no code, header, table or constant generator with
 * the HIP implementation.
 *
 * What it computes (one source at a time, in the paper's LIFO order, Sec. 2.2):
 *   - HEALPix nested ray directions, N_ray(l) = 12*4^l equal-area pixels
 *     (Sec. 2.1; pixel geometry from Gorski et al. 2005).
 *   - Each packet starts with L/N_ray(l0) and is divided equally among the four
 *     children at each split (Sec. 2.1).
 *   - Cell-by-cell segments Delta r between consecutive cell interfaces, the cell
 *     optical depth Delta tau = chi Delta r, the absorbed luminosity
 *     Delta L = L_in (1 - e^{-Delta tau}) and momentum n Delta L / c (Sec. 2.1,
 *     Eqs. e:RT2, e:Erad, e:Frad).
 *   - Splitting at r_max(l) = sqrt(3/(pi m_ray)) 2^l dx (Sec. 2.1); termination at
 *     the domain boundary or when the optical depth from the source exceeds
 *     tau_max for every frequency bin.
 *   - Opacities chi_i = n_HI sigma_H + n_H sigma_d, chi_n = n_H sigma_d (Sec. 2.3).
 *   - Photoionization rate per cell, Eq. e:photrate2: n_HI sigma_H / chi_i times
 *     the absorbed ionizing photon rate.
 *
 * Code units: dx = 1, cell volume 1, c = 1, h nu_i = 1.  Per-cell estimators:
 *   J_b[c]   = sum over segments of L_in * dr * phi(dtau),  phi(x) = (1-e^-x)/x
 *              (equals Delta L / chi exactly when chi > 0 and L_in dr in vacuum,
 *               so E_b = J_b / (c dV) is Eq. e:Erad without the 0/0 at chi = 0)
 *   force[c] = sum over bins and segments of Delta L_b * n   (chi F / c, Eq. e:radforce)
 *   rate[c]  = s_H * x_n * n_H * J_0[c]                     (Eq. e:photrate2)
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *   - a ray splits exactly at r = r_max(l), mid-cell; each child starts at r_max(l)
 *     along its own direction; split only if r_max(l) < d_exit (a tie exits);
 *   - priority within the last segment: terminate > split > exit;
 *   - termination when tau_b > tau_term for every bin, tested after the deposit;
 *   - a child whose start point lies outside the domain is created and exits
 *     with no segment (its luminosity counts as escaped);
 *   - rays at level_max never split.
 *
 * Precision: everything in double; inputs are double arrays (the tests pass the
 * exact float32 values the GPU sees).  Build with -ffp-contract=off.
 *
 * Tangent (forward-mode) and adjoint (reverse-mode) derivatives of rate and force
 * with respect to n_H and x_n hold the ray tree fixed (same splits and
 * terminations as the forward pass).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_LEVELS 16
#define ORC_MAX_BINS 2

typedef struct {
    int nx, ny, nz;
    int level0, level_max;
    double phi_c;    /* m_ray */
    double tau_term; /* terminate once tau_b > tau_term in every bin */
    double s_H;      /* gas opacity per unit n_H x_n (per cell length) */
    double s_d;      /* dust opacity per unit n_H (per cell length) */
    int n_bins;      /* 1: ionizing only; 2: ionizing + non-ionizing */
    double rot[9];   /* row-major rotation applied to every HEALPix direction */
} orc_params;

/* Per-source statistics; arrays are [n_src][ORC_MAX_LEVELS] or [n_src][ORC_MAX_BINS]. */
typedef struct {
    int64_t *created, *split, *exited, *terminated;
    int64_t *segments;                 /* [n_src] */
    double *escaped, *residual, *absorbed, *emitted;
    uint64_t destroy;                  /* sum over ended rays of 4^(level_max - level) */
} orc_stats;

/* ------------------------------------------------------------------------- */
/* HEALPix nested scheme (Gorski et al. 2005)                                */
/* ------------------------------------------------------------------------- */

/* De-interleave the bits of the within-face index: x from the even bits,
 * y from the odd bits (the nested index is a Z-order curve in each face). */
static void orc_unzip(int64_t ipf, int64_t *x, int64_t *y)
{
    int64_t xx = 0, yy = 0;
    for (int b = 0; b < 31; ++b) {
        xx |= ((ipf >> (2 * b)) & 1) << b;
        yy |= ((ipf >> (2 * b + 1)) & 1) << b;
    }
    *x = xx;
    *y = yy;
}

/* Centre (z = cos theta, phi) of nested pixel `pix` at resolution nside = 2^level.
 * Base face f has ring-row F1 = f/4 + 2 and column F2 = 2 (f mod 4) - (f/4 mod 2) + 1;
 * the ring index counted from the north pole is i = F1*nside - x - y - 1, and the
 * position in the ring follows the ring-scheme formulas for the polar caps and the
 * equatorial belt. */
void orc_pix2ang_nest(int level, int64_t pix, double *z, double *phi)
{
    const int64_t ns = (int64_t)1 << level;
    const int64_t npface = ns * ns;
    const int64_t f = pix / npface;
    int64_t x, y;
    orc_unzip(pix % npface, &x, &y);
    const int64_t F1 = f / 4 + 2;
    const int64_t F2 = 2 * (f % 4) - ((f / 4) % 2) + 1;
    const int64_t i = F1 * ns - x - y - 1; /* ring index, 1 .. 4 nside - 1 */
    int64_t nr;   /* number of pixels in the ring / 4 */
    int64_t s;    /* half-pixel shift of the ring */
    if (i < ns) {                 /* north polar cap */
        nr = i;
        *z = 1.0 - (double)(i * i) / (3.0 * (double)npface);
        s = 1;
    } else if (i > 3 * ns) {      /* south polar cap */
        nr = 4 * ns - i;
        *z = -1.0 + (double)(nr * nr) / (3.0 * (double)npface);
        s = 1;
    } else {                      /* equatorial belt */
        nr = ns;
        *z = (4.0 / 3.0) - 2.0 * (double)i / (3.0 * (double)ns);
        s = ((i - ns + 1) % 2);   /* 1 on rings aligned with the polar-cap shift */
    }
    /* in-ring position j in 1 .. 4 nr */
    int64_t j = (F2 * nr + x - y + 1 + (1 - s)) / 2;
    if (j > 4 * nr) j -= 4 * nr;
    if (j < 1) j += 4 * nr;
    *phi = (M_PI / (2.0 * (double)nr)) * ((double)j - 0.5 * (double)(2 - s));
}

void orc_pix2vec_nest(int level, int64_t pix, double v[3])
{
    double z, phi;
    orc_pix2ang_nest(level, pix, &z, &phi);
    const double st = sqrt((1.0 - z) * (1.0 + z));
    v[0] = st * cos(phi);
    v[1] = st * sin(phi);
    v[2] = z;
}

/* ------------------------------------------------------------------------- */
/* Geometry of one ray                                                        */
/* ------------------------------------------------------------------------- */

/* Splitting radius: (dx/r)^2 < m_ray Omega_ray, Omega_ray = 4 pi / (12 4^l)
 * gives r_max(l) = sqrt(3 / (pi m_ray)) 2^l  (Sec. 2.1). */
double orc_r_max(double phi_c, int level)
{
    return sqrt(3.0 / (M_PI * phi_c)) * ldexp(1.0, level);
}

static void orc_direction(const orc_params *P, int level, int64_t pix, double n[3])
{
    double v[3];
    orc_pix2vec_nest(level, pix, v);
    for (int a = 0; a < 3; ++a)
        n[a] = P->rot[3 * a + 0] * v[0] + P->rot[3 * a + 1] * v[1] + P->rot[3 * a + 2] * v[2];
}

/* Distance along n from xs to the domain boundary (slab method). */
static double orc_exit_distance(const orc_params *P, const double xs[3], const double n[3])
{
    const double hi[3] = {(double)P->nx, (double)P->ny, (double)P->nz};
    double d = INFINITY;
    for (int a = 0; a < 3; ++a) {
        double t = INFINITY;
        if (n[a] > 0.0) t = (hi[a] - xs[a]) / n[a];
        else if (n[a] < 0.0) t = (0.0 - xs[a]) / n[a];
        if (t < d) d = t;
    }
    return d;
}

typedef struct {
    int64_t cell;
    double dr;
    double dtau[ORC_MAX_BINS];
    double kappa[ORC_MAX_BINS];
} orc_seg;

typedef struct {
    orc_seg *s;
    size_t n, cap;
} orc_segbuf;

static void orc_push_seg(orc_segbuf *b, int64_t cell, double dr, const double *kappa, int nb)
{
    if (b->n == b->cap) {
        b->cap = b->cap ? 2 * b->cap : 256;
        b->s = (orc_seg *)realloc(b->s, b->cap * sizeof(orc_seg));
    }
    orc_seg *g = &b->s[b->n++];
    g->cell = cell;
    g->dr = dr;
    for (int q = 0; q < nb; ++q) {
        g->kappa[q] = kappa[q];
        g->dtau[q] = kappa[q] * dr;
    }
}

enum { ORC_EXIT = 0, ORC_SPLIT = 1, ORC_TERM = 2 };

/* Opacity per cell length of bin q in cell c (Sec. 2.3): ionizing bin sees gas
 * (n_HI sigma_H = n_H x_n s_H) plus dust (n_H s_d); the non-ionizing bin dust only. */
static double orc_kappa(const orc_params *P, const double *nH, const double *xn, int64_t c, int q)
{
    if (q == 0) return nH[c] * (xn[c] * P->s_H + P->s_d);
    return nH[c] * P->s_d;
}

/* March one ray from r_a outward, cell by cell (Amanatides-Woo style traversal:
 * the next interface along each axis, take the nearest).  Appends the segments
 * (cell, dr, kappa, dtau) to `out`, stops at the split radius, the domain exit,
 * or once every bin's optical depth from the source exceeds tau_term.
 * Returns ORC_EXIT / ORC_SPLIT / ORC_TERM; tau is updated in place. */
static int orc_march(const orc_params *P, const double *nH, const double *xn,
                     const double xs[3], const double n[3], double r_a, double r_split,
                     double d_exit, double *tau, orc_segbuf *out)
{
    const int64_t N[3] = {P->nx, P->ny, P->nz};
    const int nb = P->n_bins;
    int64_t cell[3];
    double tnext[3];
    for (int a = 0; a < 3; ++a) {
        double p = xs[a] + r_a * n[a];
        int64_t c = (int64_t)floor(p);
        if (c < 0) c = 0;
        if (c > N[a] - 1) c = N[a] - 1;
        cell[a] = c;
        if (n[a] > 0.0) tnext[a] = ((double)(c + 1) - xs[a]) / n[a];
        else if (n[a] < 0.0) tnext[a] = ((double)c - xs[a]) / n[a];
        else tnext[a] = INFINITY;
    }
    const int can_split = r_split < d_exit;
    const double r_end = can_split ? r_split : d_exit;
    double r = r_a;
    for (;;) {
        double rb = tnext[0];
        if (tnext[1] < rb) rb = tnext[1];
        if (tnext[2] < rb) rb = tnext[2];
        int ends = 0;
        if (r_end <= rb) {
            rb = r_end;
            ends = 1;
        }
        const double dr = rb - r;
        if (dr > 0.0) {
            const int64_t c = (cell[2] * N[1] + cell[1]) * N[0] + cell[0];
            double kap[ORC_MAX_BINS];
            for (int q = 0; q < nb; ++q) kap[q] = orc_kappa(P, nH, xn, c, q);
            orc_push_seg(out, c, dr, kap, nb);
            int all_thick = 1;
            for (int q = 0; q < nb; ++q) {
                tau[q] += kap[q] * dr;
                if (!(tau[q] > P->tau_term)) all_thick = 0;
            }
            if (all_thick) return ORC_TERM;
            r = rb;
        }
        if (ends) return can_split ? ORC_SPLIT : ORC_EXIT;
        for (int a = 0; a < 3; ++a) {
            if (tnext[a] == rb) {
                if (n[a] > 0.0) {
                    cell[a] += 1;
                    if (cell[a] >= N[a]) return ORC_EXIT; /* rounding guard */
                    tnext[a] = ((double)(cell[a] + 1) - xs[a]) / n[a];
                } else {
                    cell[a] -= 1;
                    if (cell[a] < 0) return ORC_EXIT;     /* rounding guard */
                    tnext[a] = ((double)cell[a] - xs[a]) / n[a];
                }
            }
        }
    }
}

/* (1 - e^{-x}) / x and its derivative, accurate for small x. */
static double orc_phi(double x)
{
    if (x == 0.0) return 1.0;
    if (fabs(x) < 1e-5) return 1.0 - x / 2.0 + x * x / 6.0;
    return -expm1(-x) / x;
}

static double orc_dphi(double x)
{
    if (fabs(x) < 1e-3) return -0.5 + x / 3.0 - x * x / 8.0 + x * x * x / 30.0;
    return (x * exp(-x) + expm1(-x)) / (x * x);
}

typedef struct {
    int level;
    int64_t pix;
    double tau[ORC_MAX_BINS];
    double dtau[ORC_MAX_BINS]; /* tangent of tau (tangent mode only) */
} orc_ray;

typedef struct {
    orc_ray *r;
    size_t n, cap;
} orc_stack;

static void orc_stack_push(orc_stack *s, orc_ray r)
{
    if (s->n == s->cap) {
        s->cap = s->cap ? 2 * s->cap : 1024;
        s->r = (orc_ray *)realloc(s->r, s->cap * sizeof(orc_ray));
    }
    s->r[s->n++] = r;
}

static int orc_check(const orc_params *P, int n_src, const double *src_pos)
{
    if (P->nx <= 0 || P->ny <= 0 || P->nz <= 0) return -1;
    if (P->level0 < 0 || P->level_max < P->level0 || P->level_max >= ORC_MAX_LEVELS) return -1;
    if (P->n_bins < 1 || P->n_bins > ORC_MAX_BINS) return -1;
    if (!(P->phi_c > 0.0)) return -1;
    for (int s = 0; s < n_src; ++s) {
        const double *x = src_pos + 3 * s;
        if (!(x[0] >= 0.0 && x[0] < P->nx && x[1] >= 0.0 && x[1] < P->ny && x[2] >= 0.0 &&
              x[2] < P->nz))
            return -2;
    }
    return 0;
}

/* Seed order of Sec. 2.2, Step 1: the 12 base-pixel trees interleaved,
 * pixel k of the sequence is (k mod 12) * 4^l0 + k / 12.  The stack is LIFO, so
 * the seeds are pushed in reverse to pop in this order. */
static void orc_seed(orc_stack *st, int level0, int n_bins)
{
    const int64_t per_face = (int64_t)1 << (2 * level0);
    const int64_t nr = 12 * per_face;
    for (int64_t k = nr - 1; k >= 0; --k) {
        orc_ray r;
        memset(&r, 0, sizeof r);
        r.level = level0;
        r.pix = (k % 12) * per_face + k / 12;
        (void)n_bins;
        orc_stack_push(st, r);
    }
}

/* ------------------------------------------------------------------------- */
/* Forward sweep                                                              */
/* ------------------------------------------------------------------------- */

/* Outputs (all overwritten):
 *   J     [n_bins][N]  mean-intensity estimator per bin (may be NULL)
 *   force [3][N]       absorbed momentum per unit time (SoA)
 *   rate  [N]          photoionizations per unit time
 * src_lum is [n_src][n_bins].  Returns 0 on success, < 0 on bad input. */
int orc_trace(const orc_params *P, const double *nH, const double *xn, int n_src,
              const double *src_pos, const double *src_lum, double *J, double *force,
              double *rate, orc_stats *st)
{
    int rc = orc_check(P, n_src, src_pos);
    if (rc) return rc;
    const int64_t N = (int64_t)P->nx * P->ny * P->nz;
    const int nb = P->n_bins;
    double *Jw = (double *)calloc((size_t)(nb * N), sizeof(double));
    memset(force, 0, sizeof(double) * 3 * N);
    orc_stack stack = {0};
    orc_segbuf segs = {0};
    if (st) st->destroy = 0;
    for (int s = 0; s < n_src; ++s) {
        const double *xs = src_pos + 3 * s;
        const double *Ls = src_lum + nb * s;
        orc_seed(&stack, P->level0, nb);
        while (stack.n) {
            orc_ray ray = stack.r[--stack.n];
            const int l = ray.level;
            double n[3];
            orc_direction(P, l, ray.pix, n);
            const double r_a = (l == P->level0) ? 0.0 : orc_r_max(P->phi_c, l - 1);
            const double r_split = (l < P->level_max) ? orc_r_max(P->phi_c, l) : INFINITY;
            const double d_exit = orc_exit_distance(P, xs, n);
            /* packet luminosity per bin: L / N_ray(l) */
            double Lnom[ORC_MAX_BINS];
            for (int q = 0; q < nb; ++q) Lnom[q] = Ls[q] / (12.0 * ldexp(1.0, 2 * l));
            if (st) st->created[s * ORC_MAX_LEVELS + l] += 1;
            int how;
            segs.n = 0;
            double tau[ORC_MAX_BINS];
            memcpy(tau, ray.tau, sizeof tau);
            if (r_a >= d_exit) {
                how = ORC_EXIT;
            } else {
                how = orc_march(P, nH, xn, xs, n, r_a, r_split, d_exit, tau, &segs);
            }
            /* deposit along the segments */
            double tin[ORC_MAX_BINS];
            memcpy(tin, ray.tau, sizeof tin);
            for (size_t k = 0; k < segs.n; ++k) {
                const orc_seg *g = &segs.s[k];
                double dLsum = 0.0;
                for (int q = 0; q < nb; ++q) {
                    const double Lin = Lnom[q] * exp(-tin[q]);
                    Jw[q * N + g->cell] += Lin * g->dr * orc_phi(g->dtau[q]);
                    const double dL = Lin * (-expm1(-g->dtau[q]));
                    dLsum += dL;
                    if (st) st->absorbed[s * ORC_MAX_BINS + q] += dL;
                    tin[q] += g->dtau[q];
                }
                force[0 * N + g->cell] += n[0] * dLsum;
                force[1 * N + g->cell] += n[1] * dLsum;
                force[2 * N + g->cell] += n[2] * dLsum;
            }
            if (st) st->segments[s] += (int64_t)segs.n;
            if (how == ORC_SPLIT) {
                if (st) st->split[s * ORC_MAX_LEVELS + l] += 1;
                for (int k = 3; k >= 0; --k) {
                    orc_ray c;
                    memset(&c, 0, sizeof c);
                    c.level = l + 1;
                    c.pix = 4 * ray.pix + k;
                    memcpy(c.tau, tau, sizeof tau);
                    orc_stack_push(&stack, c);
                }
            } else {
                if (st) {
                    if (how == ORC_EXIT) st->exited[s * ORC_MAX_LEVELS + l] += 1;
                    else st->terminated[s * ORC_MAX_LEVELS + l] += 1;
                    for (int q = 0; q < nb; ++q) {
                        const double Lleft = Lnom[q] * exp(-tau[q]);
                        if (how == ORC_EXIT) st->escaped[s * ORC_MAX_BINS + q] += Lleft;
                        else st->residual[s * ORC_MAX_BINS + q] += Lleft;
                    }
                    st->destroy += (uint64_t)1 << (2 * (P->level_max - l));
                }
            }
        }
        if (st)
            for (int q = 0; q < nb; ++q) st->emitted[s * ORC_MAX_BINS + q] = Ls[q];
    }
    for (int64_t c = 0; c < N; ++c) rate[c] = P->s_H * xn[c] * nH[c] * Jw[c];
    if (J) memcpy(J, Jw, sizeof(double) * nb * N);
    free(Jw);
    free(stack.r);
    free(segs.s);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Tangent (forward-mode derivative, tree held fixed)                         */
/* ------------------------------------------------------------------------- */

/* Directional derivative of (rate, force) along (dnH, dxn).  The ray tree
 * (splits and terminations) is that of the unperturbed forward sweep. */
int orc_tangent(const orc_params *P, const double *nH, const double *xn, const double *dnH,
                const double *dxn, int n_src, const double *src_pos, const double *src_lum,
                double *drate, double *dforce)
{
    int rc = orc_check(P, n_src, src_pos);
    if (rc) return rc;
    const int64_t N = (int64_t)P->nx * P->ny * P->nz;
    const int nb = P->n_bins;
    double *J0 = (double *)calloc((size_t)N, sizeof(double));
    double *dJ0 = (double *)calloc((size_t)N, sizeof(double));
    memset(dforce, 0, sizeof(double) * 3 * N);
    orc_stack stack = {0};
    orc_segbuf segs = {0};
    for (int s = 0; s < n_src; ++s) {
        const double *xs = src_pos + 3 * s;
        const double *Ls = src_lum + nb * s;
        orc_seed(&stack, P->level0, nb);
        while (stack.n) {
            orc_ray ray = stack.r[--stack.n];
            const int l = ray.level;
            double n[3];
            orc_direction(P, l, ray.pix, n);
            const double r_a = (l == P->level0) ? 0.0 : orc_r_max(P->phi_c, l - 1);
            const double r_split = (l < P->level_max) ? orc_r_max(P->phi_c, l) : INFINITY;
            const double d_exit = orc_exit_distance(P, xs, n);
            double Lnom[ORC_MAX_BINS];
            for (int q = 0; q < nb; ++q) Lnom[q] = Ls[q] / (12.0 * ldexp(1.0, 2 * l));
            segs.n = 0;
            double tau[ORC_MAX_BINS];
            memcpy(tau, ray.tau, sizeof tau);
            int how = ORC_EXIT;
            if (r_a < d_exit) how = orc_march(P, nH, xn, xs, n, r_a, r_split, d_exit, tau, &segs);
            double tin[ORC_MAX_BINS], dtin[ORC_MAX_BINS];
            memcpy(tin, ray.tau, sizeof tin);
            memcpy(dtin, ray.dtau, sizeof dtin);
            for (size_t k = 0; k < segs.n; ++k) {
                const orc_seg *g = &segs.s[k];
                const int64_t c = g->cell;
                /* d kappa / d inputs (Sec. 2.3 opacities) */
                double dkap[ORC_MAX_BINS];
                dkap[0] = dnH[c] * (xn[c] * P->s_H + P->s_d) + nH[c] * P->s_H * dxn[c];
                if (nb > 1) dkap[1] = dnH[c] * P->s_d;
                double ddL = 0.0;
                for (int q = 0; q < nb; ++q) {
                    const double Lin = Lnom[q] * exp(-tin[q]);
                    const double dLin = -Lin * dtin[q];
                    const double x = g->dtau[q];
                    const double ddtau = dkap[q] * g->dr;
                    if (q == 0) {
                        J0[c] += Lin * g->dr * orc_phi(x);
                        dJ0[c] += dLin * g->dr * orc_phi(x) + Lin * g->dr * orc_dphi(x) * ddtau;
                    }
                    ddL += dLin * (-expm1(-x)) + Lin * exp(-x) * ddtau;
                    tin[q] += x;
                    dtin[q] += ddtau;
                }
                dforce[0 * N + c] += n[0] * ddL;
                dforce[1 * N + c] += n[1] * ddL;
                dforce[2 * N + c] += n[2] * ddL;
            }
            if (how == ORC_SPLIT) {
                for (int k = 3; k >= 0; --k) {
                    orc_ray ch;
                    memset(&ch, 0, sizeof ch);
                    ch.level = l + 1;
                    ch.pix = 4 * ray.pix + k;
                    memcpy(ch.tau, tau, sizeof tau);
                    memcpy(ch.dtau, dtin, sizeof dtin);
                    orc_stack_push(&stack, ch);
                }
            }
        }
    }
    for (int64_t c = 0; c < N; ++c)
        drate[c] = P->s_H * (dxn[c] * nH[c] * J0[c] + xn[c] * dnH[c] * J0[c] + xn[c] * nH[c] * dJ0[c]);
    free(J0);
    free(dJ0);
    free(stack.r);
    free(segs.s);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Adjoint (reverse-mode derivative, tree held fixed)                         */
/* ------------------------------------------------------------------------- */

typedef struct {
    const orc_params *P;
    const double *nH, *xn, *w, *v, *xs, *Lsrc;
    int64_t N;
    double *gk;   /* [n_bins][N]  dL / d kappa_b per cell */
    double *J0;   /* [N]          forward J of the ionizing bin */
} orc_adj_ctx;

/* Reverse sweep of one ray and its whole subtree.  Returns, in G[b], the total
 * contribution of bin b to the loss from the ray's start point downstream
 * (its own segments plus all descendants); every such contribution is
 * proportional to e^{-tau}, so d(downstream)/d kappa_{b,k} = -dr_k * G_b(>k). */
static void orc_adj_ray(orc_adj_ctx *A, int level, int64_t pix, const double *tau0, double *G)
{
    const orc_params *P = A->P;
    const int nb = P->n_bins;
    const int64_t N = A->N;
    double n[3];
    orc_direction(P, level, pix, n);
    const double r_a = (level == P->level0) ? 0.0 : orc_r_max(P->phi_c, level - 1);
    const double r_split = (level < P->level_max) ? orc_r_max(P->phi_c, level) : INFINITY;
    const double d_exit = orc_exit_distance(P, A->xs, n);
    double Lnom[ORC_MAX_BINS];
    for (int q = 0; q < nb; ++q) Lnom[q] = A->Lsrc[q] / (12.0 * ldexp(1.0, 2 * level));
    orc_segbuf segs = {0};
    double tau[ORC_MAX_BINS] = {0.0, 0.0};
    memcpy(tau, tau0, sizeof(double) * nb);
    int how = ORC_EXIT;
    if (r_a < d_exit) how = orc_march(P, A->nH, A->xn, A->xs, n, r_a, r_split, d_exit, tau, &segs);
    double Gq[ORC_MAX_BINS] = {0.0, 0.0};
    if (how == ORC_SPLIT) {
        for (int k = 0; k < 4; ++k) {
            double Gc[ORC_MAX_BINS] = {0.0, 0.0};
            orc_adj_ray(A, level + 1, 4 * pix + k, tau, Gc);
            for (int q = 0; q < nb; ++q) Gq[q] += Gc[q];
        }
    }
    /* optical depth at the entry of each segment, then walk backwards */
    double *tin = (double *)malloc(sizeof(double) * (segs.n + 1) * ORC_MAX_BINS);
    for (int q = 0; q < nb; ++q) tin[q] = tau0[q];
    for (size_t k = 0; k < segs.n; ++k)
        for (int q = 0; q < nb; ++q)
            tin[(k + 1) * ORC_MAX_BINS + q] = tin[k * ORC_MAX_BINS + q] + segs.s[k].dtau[q];
    for (size_t kk = segs.n; kk-- > 0;) {
        const orc_seg *g = &segs.s[kk];
        const int64_t c = g->cell;
        const double a = A->w[c] * P->s_H * A->xn[c] * A->nH[c]; /* d loss / d J_0 */
        const double beta = A->v[0 * N + c] * n[0] + A->v[1 * N + c] * n[1] + A->v[2 * N + c] * n[2];
        for (int q = 0; q < nb; ++q) {
            const double Lin = Lnom[q] * exp(-tin[kk * ORC_MAX_BINS + q]);
            const double x = g->dtau[q];
            const double e = exp(-x);
            const double aq = (q == 0) ? a : 0.0;
            /* loss contributed by this segment in bin q */
            const double own = aq * Lin * g->dr * orc_phi(x) + beta * Lin * (-expm1(-x));
            /* d loss / d kappa_q of this cell through this segment */
            const double dk = aq * Lin * g->dr * g->dr * orc_dphi(x) + beta * Lin * g->dr * e
                              - g->dr * Gq[q];
            A->gk[q * N + c] += dk;
            Gq[q] += own;
        }
    }
    for (int q = 0; q < nb; ++q) G[q] = Gq[q];
    free(tin);
    free(segs.s);
}

/* Gradient of loss = sum_c w_c rate_c + sum_c v_c . force_c with respect to n_H
 * and x_n (tree held fixed).  v is [3][N] SoA.  Outputs are overwritten. */
int orc_adjoint(const orc_params *P, const double *nH, const double *xn, int n_src,
                const double *src_pos, const double *src_lum, const double *w, const double *v,
                double *g_nH, double *g_xn)
{
    int rc = orc_check(P, n_src, src_pos);
    if (rc) return rc;
    const int64_t N = (int64_t)P->nx * P->ny * P->nz;
    const int nb = P->n_bins;
    double *gk = (double *)calloc((size_t)(ORC_MAX_BINS * N), sizeof(double));
    double *J = (double *)calloc((size_t)(nb * N), sizeof(double));
    double *F = (double *)calloc((size_t)(3 * N), sizeof(double));
    double *R = (double *)calloc((size_t)N, sizeof(double));
    orc_trace(P, nH, xn, n_src, src_pos, src_lum, J, F, R, NULL);
    orc_adj_ctx A = {P, nH, xn, w, v, NULL, NULL, N, gk, J};
    const int64_t per_face = (int64_t)1 << (2 * P->level0);
    for (int s = 0; s < n_src; ++s) {
        A.xs = src_pos + 3 * s;
        A.Lsrc = src_lum + nb * s;
        for (int64_t p = 0; p < 12 * per_face; ++p) {
            double tau0[ORC_MAX_BINS] = {0.0, 0.0};
            double G[ORC_MAX_BINS];
            orc_adj_ray(&A, P->level0, p, tau0, G);
        }
    }
    /* chain rule through kappa_0 = n_H (x_n s_H + s_d), kappa_1 = n_H s_d,
     * plus the explicit n_H x_n factor of rate = s_H x_n n_H J_0 */
    for (int64_t c = 0; c < N; ++c) {
        const double d1 = (nb > 1) ? gk[N + c] * P->s_d : 0.0;
        g_nH[c] = gk[c] * (xn[c] * P->s_H + P->s_d) + d1 + w[c] * P->s_H * xn[c] * J[c];
        g_xn[c] = gk[c] * nH[c] * P->s_H + w[c] * P->s_H * nH[c] * J[c];
    }
    free(gk);
    free(J);
    free(F);
    free(R);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* Small helpers exposed for the pin tests                                    */
/* ------------------------------------------------------------------------- */

/* The first n pixels of the level-l0 seed sequence in the order the stack pops
 * them (Sec. 2.2, Step 1); returns how many were written. */
int64_t orc_seed_order(int level0, int64_t *pix, int64_t n)
{
    orc_stack st = {0};
    orc_seed(&st, level0, 1);
    int64_t k = 0;
    while (st.n && k < n) pix[k++] = st.r[--st.n].pix;
    free(st.r);
    return k;
}

/* Segments of a single ray from (xs, n) over [r_a, r_end] through a grid with
 * zero opacity: writes up to `cap` (cell, dr) pairs and returns the count
 * (or -count when truncated).  Used by the traversal pin test. */
int64_t orc_ray_segments(int nx, int ny, int nz, const double xs[3], const double n[3],
                         double r_a, double r_end, int64_t *cells, double *drs, int64_t cap)
{
    orc_params P;
    memset(&P, 0, sizeof P);
    P.nx = nx;
    P.ny = ny;
    P.nz = nz;
    P.n_bins = 1;
    P.tau_term = INFINITY;
    P.rot[0] = P.rot[4] = P.rot[8] = 1.0;
    const double d_exit = orc_exit_distance(&P, xs, n);
    if (r_a >= d_exit) return 0;
    double *zero = (double *)calloc((size_t)nx * ny * nz, sizeof(double));
    double tau[ORC_MAX_BINS] = {0.0, 0.0};
    orc_segbuf segs = {0};
    orc_march(&P, zero, zero, xs, n, r_a, r_end, d_exit, tau, &segs);
    int64_t m = (int64_t)segs.n;
    for (int64_t k = 0; k < m && k < cap; ++k) {
        cells[k] = segs.s[k].cell;
        drs[k] = segs.s[k].dr;
    }
    free(zero);
    free(segs.s);
    return m <= cap ? m : -m;
}
