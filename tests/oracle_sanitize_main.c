/* Drives the FP64 oracle (compiled into this program) on a small problem so that
 * the CPU test suite can run it under AddressSanitizer and UndefinedBehaviorSanitizer:
 * forward trace, tangent and adjoint of a 2-bin lognormal-like field with three
 * sources, plus a source outside the box (rejected).  Exits 0 when every call
 * returns its expected code and photons are conserved. */
#include "../oracle/art_oracle.c"

#include <stdio.h>
#include <stdlib.h>

int main(void)
{
    const int n = 14, N = n * n * n, ns = 3;
    orc_params P;
    memset(&P, 0, sizeof P);
    P.nx = P.ny = P.nz = n;
    P.level0 = 2;
    P.level_max = 13;
    P.phi_c = 4.0;
    P.tau_term = 23.025850929940457;
    P.s_H = 0.3;
    P.s_d = 0.03;
    P.n_bins = 2;
    P.rot[0] = P.rot[4] = P.rot[8] = 1.0;
    double *nH = malloc(sizeof(double) * N), *xn = malloc(sizeof(double) * N);
    double *J = calloc(2 * (size_t)N, sizeof(double)), *F = calloc(3 * (size_t)N, sizeof(double));
    double *rate = calloc(N, sizeof(double)), *w = malloc(sizeof(double) * N), *v = malloc(sizeof(double) * 3 * N);
    double *g1 = calloc(N, sizeof(double)), *g2 = calloc(N, sizeof(double));
    for (int i = 0; i < N; ++i) {
        nH[i] = exp(sin(0.37 * i) + 0.5 * cos(0.011 * i * i));
        xn[i] = 0.5 + 0.5 * sin(0.13 * i);
        w[i] = 0.5 + 0.4 * cos(0.7 * i);
        v[i] = 0.1 * sin(i);
        v[N + i] = 0.2 * cos(i);
        v[2 * N + i] = 0.3;
    }
    const double pos[9] = {7.2, 6.9, 7.4, 2.1, 11.3, 5.5, 12.9, 0.4, 9.9};
    const double lum[6] = {1.0, 1.5, 30.0, 45.0, 0.2, 0.3};
    int64_t created[3 * ORC_MAX_LEVELS], split[3 * ORC_MAX_LEVELS], exited[3 * ORC_MAX_LEVELS],
        term[3 * ORC_MAX_LEVELS], segs[3];
    double esc[3 * ORC_MAX_BINS], res[3 * ORC_MAX_BINS], abs_[3 * ORC_MAX_BINS], emit[3 * ORC_MAX_BINS];
    orc_stats S = {created, split, exited, term, segs, esc, res, abs_, emit, 0};
    int rc = orc_trace(&P, nH, xn, ns, pos, lum, J, F, rate, &S);
    if (rc != 0) { fprintf(stderr, "trace rc %d\n", rc); return 1; }
    for (int b = 0; b < 2; ++b) {
        double a = 0.0, e = 0.0, out = 0.0;
        for (int s = 0; s < ns; ++s) {
            a += abs_[s * ORC_MAX_BINS + b];
            e += emit[s * ORC_MAX_BINS + b];
            out += esc[s * ORC_MAX_BINS + b] + res[s * ORC_MAX_BINS + b];
        }
        if (fabs(a + out - e) > 1e-10 * e) { fprintf(stderr, "conservation bin %d\n", b); return 1; }
    }
    if (S.destroy != (uint64_t)ns * (12ull << 26)) { fprintf(stderr, "destroy count\n"); return 1; }
    double *dr = calloc(N, sizeof(double)), *df = calloc(3 * (size_t)N, sizeof(double));
    rc = orc_tangent(&P, nH, xn, w, xn, ns, pos, lum, dr, df);
    if (rc != 0) { fprintf(stderr, "tangent rc %d\n", rc); return 1; }
    rc = orc_adjoint(&P, nH, xn, ns, pos, lum, w, v, g1, g2);
    if (rc != 0) { fprintf(stderr, "adjoint rc %d\n", rc); return 1; }
    const double outside[3] = {7.0, 7.0, (double)n + 1.0};
    if (orc_trace(&P, nH, xn, 1, outside, lum, J, F, rate, &S) == 0) { fprintf(stderr, "outside accepted\n"); return 1; }
    free(nH); free(xn); free(J); free(F); free(rate); free(w); free(v); free(g1); free(g2); free(dr); free(df);
    puts("oracle sanitize run: ok");
    return 0;
}
