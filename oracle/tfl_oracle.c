/*
 * tfl_oracle.c -- plain FP64 CPU oracle of the two-fluid (Maxwell + London)
 * FDTD scheme.
 *
 * TEST INFRASTRUCTURE ONLY.  It is built into oracle/liboracle.so and is
 * loaded by tests/, by the smoke check and by the CPU-baseline leg of the
 * benchmark.  The product library never links, loads or calls it, and the
 * two share no source, header or table.
 *
 * What it computes (paper: Sec. 2 Eqs. Ampere, Faraday, London1a; Sec. 3 and
 * Algorithm 1):
 *   State at integer time n: E^n on cell edges, B^n on cell faces, Js^n on
 *   the superconducting cell edges (Yee staggering, Sec. 3).  One time step is
 *   the five sub-steps of Algorithm 1 in the paper's order:
 *     1. B^{n+1/2}  = B^n - dt/2 curl E^n
 *     2. Js^{n+1/2} = Js^n + dt/2 * E^n / (lambda^2 mu0)        (SC edges only)
 *     3. E^{n+1}    = (1 + theta s)^-1 (E^n + dt/eps curl H^{n+1/2}
 *                      - (1 - theta) s E^n - dt/eps Js^{n+1/2}),  s = sigma dt/eps
 *     4. Js^{n+1}   = Js^{n+1/2} + dt/2 * E^{n+1} / (lambda^2 mu0)
 *     5. B^{n+1}    = B^{n+1/2} - dt/2 curl E^{n+1}
 *   with H = B / mu0 (mu_r = 1, Sec. 4.2 and Sec. 5).
 *
 * Readings where the paper is silent (each is listed in the design notes):
 *   - per-edge material: an edge whose four sharing cells include any
 *     superconducting cell (ell > 0) is superconducting and takes the mean of
 *     (eps_r, sigma, ell) over those superconducting cells; any other edge takes
 *     the mean of (eps_r, sigma) over all four cells and ell = 0 (Sec. 3: every
 *     edge on an SC interface is superconducting and carries Js; this choice
 *     reproduces the first-order strip errors of Table 4);
 *   - open boundaries: convolutional PML (Roden and Gedney 2000) with a
 *     polynomial grading, backed by a PEC wall on node plane 0 of every PML
 *     axis (tangential E held at 0); indexing wraps on every axis;
 *   - the PML auxiliary variable of the B update is advanced whenever a new E
 *     is available (at initialisation and in sub-step 5), so that sub-steps 1
 *     and 5 use the same stretched curl;
 *   - soft sources add A g(t_{n+1}) to E^{n+1} at the end of sub-step 3;
 *   - probes sum E over an index box; series index n holds time level n,
 *     sample 0 is the state passed to oracle_set_fields.
 *
 * The code favours plain loops over speed: every array is a full grid and
 * every neighbour index is wrapped explicitly.  The grid sweeps are split over
 * z-planes (or elements) with OpenMP when there are several; each element is
 * written by one thread from values no thread writes in the same loop, so the
 * results do not depend on the thread count.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define O_EPS0 8.8541878128e-12
#define O_MU0 1.25663706212e-6

#define O_MAXSRC 64
#define O_MAXPROBE 64

typedef struct {
    int comp;
    long box[6]; /* i0 i1 j0 j1 k0 k1, half-open, edge indices of the component */
    double amp;
    int kind;    /* 0 sin(2 pi f t), 1 gauss, 2 gauss * sin(2 pi f t) */
    double f, t0, tw;
} o_source;

typedef struct {
    int comp;
    long box[6];
    long cap;
    double *series;
    int nfreq;
    double *freq;
    double *dft_re, *dft_im;
} o_probe;

typedef struct {
    long n[3];
    double d[3];
    double dt, theta;
    int pml[3];
    long npml_lo[3], npml_hi[3];
    double pml_order, pml_scale, kappa_max, alpha_max;

    double *eps[3], *sig[3], *ell[3]; /* per edge of component c */
    double *cell_ell;                 /* per-cell 1/lambda^2 (classification of edges) */
    double *E[3], *B[3], *J[3];
    double *psiB[3][3]; /* [component][derivative axis] */
    double *psiE[3][3];
    /* 1-D PML coefficients per axis: at nodes (integer) and at half nodes */
    double *bn[3], *cn[3], *kin[3];
    double *bh[3], *ch[3], *kih[3];

    long step;
    int sampled0;
    int nsrc;
    o_source src[O_MAXSRC];
    int nprobe;
    o_probe probe[O_MAXPROBE];
} oracle_sim;

/* Index wrap onto [0, n): the stencils step at most one cell past an end, so
 * those cases are tested first; any other index takes the general modulo. */
static long o_wrap(long i, long n)
{
    if (i >= 0 && i < n) return i;
    if (i == -1) return n - 1;
    if (i == n) return 0;
    long r = i % n;
    return r < 0 ? r + n : r;
}

static long o_idx(const oracle_sim *s, long i, long j, long k)
{
    return (o_wrap(k, s->n[2]) * s->n[1] + o_wrap(j, s->n[1])) * s->n[0] + o_wrap(i, s->n[0]);
}

static long o_cells(const oracle_sim *s) { return s->n[0] * s->n[1] * s->n[2]; }

static double *o_zeros(long m) { return (double *)calloc((size_t)m, sizeof(double)); }

/* Position of a component's sample along an axis is half-integer when the
 * component is E and the axis is its own direction, or when the component is
 * B and the axis is not its own direction. */

/* ---- convolutional PML profile (Roden and Gedney 2000) ------------------ */
static void o_pml_coeffs(const oracle_sim *s, int ax, double pos, double *b, double *c, double *kinv)
{
    double depth = -1.0;
    long n = s->n[ax];
    long lo = s->npml_lo[ax], hi = s->npml_hi[ax];
    *b = 1.0; *c = 0.0; *kinv = 1.0;
    if (!s->pml[ax]) return;
    if (lo > 0 && pos < (double)lo) depth = ((double)lo - pos) / (double)lo;
    else if (hi > 0 && pos > (double)(n - hi)) depth = (pos - (double)(n - hi)) / (double)hi;
    if (depth <= 0.0) return;
    double eta0 = sqrt(O_MU0 / O_EPS0);
    double m = s->pml_order;
    double smax = s->pml_scale * 0.8 * (m + 1.0) / (eta0 * s->d[ax]);
    double sg = smax * pow(depth, m);
    double kp = 1.0 + (s->kappa_max - 1.0) * pow(depth, m);
    double al = s->alpha_max * (1.0 - depth);
    *b = exp(-(sg / kp + al) * s->dt / O_EPS0);
    *c = (sg > 0.0) ? sg / (sg * kp + kp * kp * al) * (*b - 1.0) : 0.0;
    *kinv = 1.0 / kp;
}

oracle_sim *oracle_create(const long *n, const double *d, double dt, double theta,
                          const int *pml, const long *npml_lo, const long *npml_hi,
                          double pml_order, double pml_scale, double kappa_max, double alpha_max)
{
    oracle_sim *s = (oracle_sim *)calloc(1, sizeof(oracle_sim));
    for (int a = 0; a < 3; ++a) {
        s->n[a] = n[a]; s->d[a] = d[a];
        s->pml[a] = pml[a]; s->npml_lo[a] = npml_lo[a]; s->npml_hi[a] = npml_hi[a];
    }
    s->dt = dt; s->theta = theta;
    s->pml_order = pml_order; s->pml_scale = pml_scale;
    s->kappa_max = kappa_max; s->alpha_max = alpha_max;
    long N = o_cells(s);
    for (int c = 0; c < 3; ++c) {
        s->eps[c] = o_zeros(N); s->sig[c] = o_zeros(N); s->ell[c] = o_zeros(N);
        s->E[c] = o_zeros(N); s->B[c] = o_zeros(N); s->J[c] = o_zeros(N);
        for (int a = 0; a < 3; ++a) {
            if (a != c && pml[a]) { s->psiB[c][a] = o_zeros(N); s->psiE[c][a] = o_zeros(N); }
        }
    }
    for (int a = 0; a < 3; ++a) {
        long m = n[a];
        s->bn[a] = o_zeros(m); s->cn[a] = o_zeros(m); s->kin[a] = o_zeros(m);
        s->bh[a] = o_zeros(m); s->ch[a] = o_zeros(m); s->kih[a] = o_zeros(m);
        for (long i = 0; i < m; ++i) {
            o_pml_coeffs(s, a, (double)i, &s->bn[a][i], &s->cn[a][i], &s->kin[a][i]);
            o_pml_coeffs(s, a, (double)i + 0.5, &s->bh[a][i], &s->ch[a][i], &s->kih[a][i]);
        }
    }
    return s;
}

void oracle_destroy(oracle_sim *s)
{
    if (!s) return;
    for (int c = 0; c < 3; ++c) {
        free(s->eps[c]); free(s->sig[c]); free(s->ell[c]);
        free(s->E[c]); free(s->B[c]); free(s->J[c]);
        for (int a = 0; a < 3; ++a) { free(s->psiB[c][a]); free(s->psiE[c][a]); }
    }
    for (int a = 0; a < 3; ++a) {
        free(s->bn[a]); free(s->cn[a]); free(s->kin[a]);
        free(s->bh[a]); free(s->ch[a]); free(s->kih[a]);
    }
    free(s->cell_ell);
    for (int p = 0; p < s->nprobe; ++p) {
        free(s->probe[p].series); free(s->probe[p].freq);
        free(s->probe[p].dft_re); free(s->probe[p].dft_im);
    }
    free(s);
}

/* Per-edge material.  An edge of component c at index (i,j,k) runs along
 * axis c; the four cells sharing it are offset by 0 or -1 along each of the
 * two other axes.  If any of them is superconducting (ell > 0) the edge is
 * superconducting and takes the mean over the superconducting ones;
 * otherwise it takes the mean over all four. */
void oracle_set_materials(oracle_sim *s, const double *eps_r, const double *sigma, const double *ell)
{
    if (!s->cell_ell) s->cell_ell = o_zeros(o_cells(s));
    memcpy(s->cell_ell, ell, (size_t)o_cells(s) * sizeof(double));
    for (int c = 0; c < 3; ++c) {
        int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
        for (long k = 0; k < s->n[2]; ++k)
            for (long j = 0; j < s->n[1]; ++j)
                for (long i = 0; i < s->n[0]; ++i) {
                    long e = o_idx(s, i, j, k);
                    long cells[4];
                    int nsc = 0;
                    for (int u = 0; u < 2; ++u)
                        for (int v = 0; v < 2; ++v) {
                            long o[3] = {i, j, k};
                            o[a1] -= u;
                            o[a2] -= v;
                            cells[2 * u + v] = o_idx(s, o[0], o[1], o[2]);
                            if (ell[cells[2 * u + v]] > 0.0) nsc += 1;
                        }
                    double se = 0.0, ss = 0.0, sl = 0.0;
                    int cnt = 0;
                    for (int q = 0; q < 4; ++q) {
                        long cc = cells[q];
                        if (nsc > 0 && !(ell[cc] > 0.0)) continue;
                        se += eps_r[cc]; ss += sigma[cc]; sl += ell[cc];
                        cnt += 1;
                    }
                    s->eps[c][e] = O_EPS0 * se / (double)cnt;
                    s->sig[c][e] = ss / (double)cnt;
                    s->ell[c][e] = sl / (double)cnt;
                }
    }
}

/* Is the edge of component c at (i,j,k) on the PEC wall (node plane 0 of a
 * PML axis that is not the edge's own direction)? */
static int o_on_wall(const oracle_sim *s, int c, const long *ijk)
{
    for (int a = 0; a < 3; ++a)
        if (a != c && s->pml[a] && ijk[a] == 0) return 1;
    return 0;
}

/* Stretched derivative of F along axis a at a B_c sample: forward difference.
 * Advances the PML variable first when advance != 0. */
static double o_dB(oracle_sim *s, int c, int a, const double *F, const long *ijk, long e, int advance)
{
    long p[3] = {ijk[0], ijk[1], ijk[2]};
    p[a] += 1;
    double dF = (F[o_idx(s, p[0], p[1], p[2])] - F[e]) / s->d[a];
    long ia = ijk[a];
    double val = s->kih[a][ia] * dF;
    if (s->psiB[c][a]) {
        if (advance) s->psiB[c][a][e] = s->bh[a][ia] * s->psiB[c][a][e] + s->ch[a][ia] * dF;
        val += s->psiB[c][a][e];
    }
    return val;
}

/* curl E at B_c samples, with PML stretching (Faraday's law, Eq. Faraday). */
static double o_curlE(oracle_sim *s, int c, const long *ijk, long e, int advance)
{
    int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
    /* (curl E)_c = d_{a1} E_{a2} - d_{a2} E_{a1} */
    return o_dB(s, c, a1, s->E[a2], ijk, e, advance) - o_dB(s, c, a2, s->E[a1], ijk, e, advance);
}

static void o_half_B(oracle_sim *s, int advance_psi)
{
    double h = 0.5 * s->dt;
    for (int c = 0; c < 3; ++c) {
#pragma omp parallel for if (s->n[2] > 1)
        for (long k = 0; k < s->n[2]; ++k)
            for (long j = 0; j < s->n[1]; ++j)
                for (long i = 0; i < s->n[0]; ++i) {
                    long ijk[3] = {i, j, k};
                    long e = o_idx(s, i, j, k);
                    double cE = o_curlE(s, c, ijk, e, advance_psi);
                    s->B[c][e] -= h * cE;
                }
    }
}

/* Advance only the PML variables of the B update with the current E. */
static void o_advance_psiB(oracle_sim *s)
{
    for (int c = 0; c < 3; ++c) {
#pragma omp parallel for if (s->n[2] > 1)
        for (long k = 0; k < s->n[2]; ++k)
            for (long j = 0; j < s->n[1]; ++j)
                for (long i = 0; i < s->n[0]; ++i) {
                    long ijk[3] = {i, j, k};
                    long e = o_idx(s, i, j, k);
                    (void)o_curlE(s, c, ijk, e, 1);
                }
    }
}

static void o_half_J(oracle_sim *s)
{
    for (int c = 0; c < 3; ++c) {
        long N = o_cells(s);
#pragma omp parallel for if (N > 65536)
        for (long e = 0; e < N; ++e) {
            if (s->ell[c][e] > 0.0) /* superconducting edges only */
                s->J[c][e] += 0.5 * s->dt * s->E[c][e] * s->ell[c][e] / O_MU0;
        }
    }
}

static double o_dE(oracle_sim *s, int c, int a, const double *F, const long *ijk, long e)
{
    long p[3] = {ijk[0], ijk[1], ijk[2]};
    p[a] -= 1;
    double dF = (F[e] - F[o_idx(s, p[0], p[1], p[2])]) / s->d[a];
    long ia = ijk[a];
    double val = s->kin[a][ia] * dF;
    if (s->psiE[c][a]) {
        s->psiE[c][a][e] = s->bn[a][ia] * s->psiE[c][a][e] + s->cn[a][ia] * dF;
        val += s->psiE[c][a][e];
    }
    return val;
}

static double o_waveform(const o_source *q, double t)
{
    const double twopi = 2.0 * 3.14159265358979323846;
    switch (q->kind) {
    case 0: return sin(twopi * q->f * t);
    case 1: return exp(-(t - q->t0) * (t - q->t0) / (2.0 * q->tw * q->tw));
    default: return exp(-(t - q->t0) * (t - q->t0) / (2.0 * q->tw * q->tw)) * sin(twopi * q->f * t);
    }
}

static void o_full_E(oracle_sim *s)
{
    double dt = s->dt, th = s->theta;
    /* H^{n+1/2} = B^{n+1/2} / mu0, formed once so that the curl reads H. */
    long N = o_cells(s);
    double *H[3];
    for (int c = 0; c < 3; ++c) {
        H[c] = (double *)malloc((size_t)N * sizeof(double));
#pragma omp parallel for if (N > 65536)
        for (long e = 0; e < N; ++e) H[c][e] = s->B[c][e] / O_MU0;
    }
    for (int c = 0; c < 3; ++c) {
        int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
#pragma omp parallel for if (s->n[2] > 1)
        for (long k = 0; k < s->n[2]; ++k)
            for (long j = 0; j < s->n[1]; ++j)
                for (long i = 0; i < s->n[0]; ++i) {
                    long ijk[3] = {i, j, k};
                    long e = o_idx(s, i, j, k);
                    /* (curl H)_c = d_{a1} H_{a2} - d_{a2} H_{a1} (Eq. Ampere) */
                    double cH = o_dE(s, c, a1, H[a2], ijk, e) - o_dE(s, c, a2, H[a1], ijk, e);
                    if (o_on_wall(s, c, ijk)) { s->E[c][e] = 0.0; continue; }
                    double eps = s->eps[c][e];
                    double sg = s->sig[c][e] * dt / eps;
                    double js = (s->ell[c][e] > 0.0) ? s->J[c][e] : 0.0;
                    double En = s->E[c][e];
                    s->E[c][e] = (En + dt / eps * cH - (1.0 - th) * sg * En - dt / eps * js) / (1.0 + th * sg);
                }
    }
    for (int c = 0; c < 3; ++c) free(H[c]);
    /* soft sources at t_{n+1} */
    double t = (double)(s->step + 1) * dt;
    for (int q = 0; q < s->nsrc; ++q) {
        const o_source *src = &s->src[q];
        double g = src->amp * o_waveform(src, t);
        for (long k = src->box[4]; k < src->box[5]; ++k)
            for (long j = src->box[2]; j < src->box[3]; ++j)
                for (long i = src->box[0]; i < src->box[1]; ++i)
                    s->E[src->comp][o_idx(s, i, j, k)] += g;
    }
}

static void o_sample(oracle_sim *s, long n)
{
    const double twopi = 2.0 * 3.14159265358979323846;
    for (int p = 0; p < s->nprobe; ++p) {
        o_probe *q = &s->probe[p];
        double sum = 0.0;
        for (long k = q->box[4]; k < q->box[5]; ++k)
            for (long j = q->box[2]; j < q->box[3]; ++j)
                for (long i = q->box[0]; i < q->box[1]; ++i)
                    sum += s->E[q->comp][o_idx(s, i, j, k)];
        if (n < q->cap) q->series[n] = sum;
        for (int f = 0; f < q->nfreq; ++f) {
            double ph = twopi * q->freq[f] * (double)n * s->dt;
            q->dft_re[f] += sum * s->dt * cos(ph);
            q->dft_im[f] -= sum * s->dt * sin(ph);
        }
    }
}

/* Integer-time state at t = 0.  Resets the step counter, the PML variables
 * and the probe accumulators. */
void oracle_set_fields(oracle_sim *s, double *const *E, double *const *B, double *const *J)
{
    long N = o_cells(s);
    for (int c = 0; c < 3; ++c) {
        memcpy(s->E[c], E[c], (size_t)N * sizeof(double));
        memcpy(s->B[c], B[c], (size_t)N * sizeof(double));
        memcpy(s->J[c], J[c], (size_t)N * sizeof(double));
        for (int a = 0; a < 3; ++a) {
            if (s->psiB[c][a]) memset(s->psiB[c][a], 0, (size_t)N * sizeof(double));
            if (s->psiE[c][a]) memset(s->psiE[c][a], 0, (size_t)N * sizeof(double));
        }
    }
    s->step = 0;
    s->sampled0 = 0;
    for (int p = 0; p < s->nprobe; ++p) {
        o_probe *q = &s->probe[p];
        memset(q->series, 0, (size_t)q->cap * sizeof(double));
        memset(q->dft_re, 0, (size_t)q->nfreq * sizeof(double));
        memset(q->dft_im, 0, (size_t)q->nfreq * sizeof(double));
    }
    o_advance_psiB(s);
}

void oracle_get_fields(const oracle_sim *s, double *const *E, double *const *B, double *const *J)
{
    long N = o_cells(s);
    for (int c = 0; c < 3; ++c) {
        if (E) memcpy(E[c], s->E[c], (size_t)N * sizeof(double));
        if (B) memcpy(B[c], s->B[c], (size_t)N * sizeof(double));
        if (J) memcpy(J[c], s->J[c], (size_t)N * sizeof(double));
    }
}

void oracle_get_edge_materials(const oracle_sim *s, double *const *eps, double *const *sig, double *const *ell)
{
    long N = o_cells(s);
    for (int c = 0; c < 3; ++c) {
        memcpy(eps[c], s->eps[c], (size_t)N * sizeof(double));
        memcpy(sig[c], s->sig[c], (size_t)N * sizeof(double));
        memcpy(ell[c], s->ell[c], (size_t)N * sizeof(double));
    }
}

int oracle_add_source(oracle_sim *s, int comp, const long *box, double amp, int kind, double f, double t0, double tw)
{
    if (s->nsrc >= O_MAXSRC) return -1;
    o_source *q = &s->src[s->nsrc];
    q->comp = comp;
    for (int i = 0; i < 6; ++i) q->box[i] = box[i];
    q->amp = amp; q->kind = kind; q->f = f; q->t0 = t0; q->tw = tw;
    return s->nsrc++;
}

int oracle_add_probe(oracle_sim *s, int comp, const long *box, long cap, int nfreq, const double *freq)
{
    if (s->nprobe >= O_MAXPROBE) return -1;
    o_probe *q = &s->probe[s->nprobe];
    q->comp = comp;
    for (int i = 0; i < 6; ++i) q->box[i] = box[i];
    q->cap = cap;
    q->series = o_zeros(cap > 0 ? cap : 1);
    q->nfreq = nfreq;
    q->freq = o_zeros(nfreq > 0 ? nfreq : 1);
    for (int f = 0; f < nfreq; ++f) q->freq[f] = freq[f];
    q->dft_re = o_zeros(nfreq > 0 ? nfreq : 1);
    q->dft_im = o_zeros(nfreq > 0 ? nfreq : 1);
    return s->nprobe++;
}

void oracle_probe_read(const oracle_sim *s, int p, double *series, double *dft_re, double *dft_im)
{
    const o_probe *q = &s->probe[p];
    if (series) memcpy(series, q->series, (size_t)q->cap * sizeof(double));
    if (dft_re) memcpy(dft_re, q->dft_re, (size_t)q->nfreq * sizeof(double));
    if (dft_im) memcpy(dft_im, q->dft_im, (size_t)q->nfreq * sizeof(double));
}

/* Algorithm 1, nsteps times. */
void oracle_step(oracle_sim *s, long nsteps)
{
    if (!s->sampled0 && s->step == 0) { o_sample(s, 0); s->sampled0 = 1; }
    for (long it = 0; it < nsteps; ++it) {
        o_half_B(s, 0);   /* 1. B^n -> B^{n+1/2} */
        o_half_J(s);      /* 2. Js^n -> Js^{n+1/2} */
        o_full_E(s);      /* 3. E^n -> E^{n+1} (+ soft sources) */
        o_half_J(s);      /* 4. Js^{n+1/2} -> Js^{n+1} */
        o_half_B(s, 1);   /* 5. B^{n+1/2} -> B^{n+1} (PML variable advanced with E^{n+1}) */
        s->step += 1;
        o_sample(s, s->step);
    }
}

long oracle_step_index(const oracle_sim *s) { return s->step; }

/* Threads the grid sweeps run on (1 without OpenMP). */
int oracle_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Discrete energy at integer time n, written with the integer-time state:
 *   W^n = dV [ sum_e eps_e E_e^2 / 2
 *            + sum_f (B_f^2 - (dt/2 curlE_f)^2) / (2 mu0)
 *            + sum_{SC e} mu0 (J_e^2 - (dt/2 ell_e E_e / mu0)^2) / (2 ell_e) ].
 * This equals dV [eps E^2/2 + mu0 H^{n-1/2} H^{n+1/2}/2 + mu0 J^{n-1/2} J^{n+1/2}/(2 ell)],
 * the quantity conserved by the leap-frog of Algorithm 1 without loss (and
 * decreased by exactly the Ohmic work with sigma > 0).  PML stretching is
 * ignored: meaningful on periodic domains only. */
double oracle_energy(const oracle_sim *s)
{
    double dV = s->d[0] * s->d[1] * s->d[2];
    double we = 0.0, wb = 0.0, wj = 0.0;
    long N = o_cells(s);
    for (int c = 0; c < 3; ++c) {
        int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
        for (long k = 0; k < s->n[2]; ++k)
            for (long j = 0; j < s->n[1]; ++j)
                for (long i = 0; i < s->n[0]; ++i) {
                    long e = o_idx(s, i, j, k);
                    long p1[3] = {i, j, k}, p2[3] = {i, j, k};
                    p1[a1] += 1;
                    p2[a2] += 1;
                    double cE = (s->E[a2][o_idx(s, p1[0], p1[1], p1[2])] - s->E[a2][e]) / s->d[a1]
                              - (s->E[a1][o_idx(s, p2[0], p2[1], p2[2])] - s->E[a1][e]) / s->d[a2];
                    double hb = 0.5 * s->dt * cE;
                    wb += (s->B[c][e] * s->B[c][e] - hb * hb) / (2.0 * O_MU0);
                }
        for (long e = 0; e < N; ++e) {
            we += s->eps[c][e] * s->E[c][e] * s->E[c][e] / 2.0;
            if (s->ell[c][e] > 0.0) {
                double hj = 0.5 * s->dt * s->ell[c][e] * s->E[c][e] / O_MU0;
                wj += O_MU0 * (s->J[c][e] * s->J[c][e] - hj * hj) / (2.0 * s->ell[c][e]);
            }
        }
    }
    return dV * (we + wb + wj);
}

/* ======================================================================
 * Adjoint (reverse-mode) of the run above, for the probe DFT objective
 *   J = |F|^2,  F = sum_{n=0}^{N} w_n s_n,  w_n = dt exp(-i 2 pi f0 n dt),
 * where s_n is the sample of probe `pid` (sum of E_comp over its box).
 * The forward states of every step are stored (small grids only); each
 * sub-step of Algorithm 1 is then transposed in reverse order.  Gradients
 * are taken with respect to the per-cell maps ell = 1/lambda^2 and sigma,
 * holding each edge's superconducting / normal classification fixed (the
 * derivative of the per-edge rule: weight 1/|S| over the superconducting
 * cells S of a superconducting edge, 1/4 over all cells of a normal edge).
 * ====================================================================== */

typedef struct {
    double *E[3], *B[3], *J[3];
    double *psiB[3][3], *psiE[3][3];
} o_state;

static void o_state_alloc(const oracle_sim *s, o_state *st)
{
    long N = o_cells(s);
    for (int c = 0; c < 3; ++c) {
        st->E[c] = o_zeros(N); st->B[c] = o_zeros(N); st->J[c] = o_zeros(N);
        for (int a = 0; a < 3; ++a) {
            st->psiB[c][a] = s->psiB[c][a] ? o_zeros(N) : NULL;
            st->psiE[c][a] = s->psiE[c][a] ? o_zeros(N) : NULL;
        }
    }
}

static void o_state_free(o_state *st)
{
    for (int c = 0; c < 3; ++c) {
        free(st->E[c]); free(st->B[c]); free(st->J[c]);
        for (int a = 0; a < 3; ++a) { free(st->psiB[c][a]); free(st->psiE[c][a]); }
    }
}

static void o_state_copy(const oracle_sim *s, o_state *dst, double *const *E, double *const *B, double *const *J,
                         double *const (*psiB)[3], double *const (*psiE)[3])
{
    size_t bytes = (size_t)o_cells(s) * sizeof(double);
    for (int c = 0; c < 3; ++c) {
        memcpy(dst->E[c], E[c], bytes); memcpy(dst->B[c], B[c], bytes); memcpy(dst->J[c], J[c], bytes);
        for (int a = 0; a < 3; ++a) {
            if (dst->psiB[c][a]) memcpy(dst->psiB[c][a], psiB[c][a], bytes);
            if (dst->psiE[c][a]) memcpy(dst->psiE[c][a], psiE[c][a], bytes);
        }
    }
}

static void o_state_load(oracle_sim *s, const o_state *src)
{
    o_state tmp;
    for (int c = 0; c < 3; ++c) {
        tmp.E[c] = s->E[c]; tmp.B[c] = s->B[c]; tmp.J[c] = s->J[c];
        for (int a = 0; a < 3; ++a) { tmp.psiB[c][a] = s->psiB[c][a]; tmp.psiE[c][a] = s->psiE[c][a]; }
    }
    o_state_copy(s, &tmp, src->E, src->B, src->J, src->psiB, src->psiE);
}

static double o_probe_sum(const oracle_sim *s, int comp, const long *box)
{
    double sum = 0.0;
    for (long k = box[4]; k < box[5]; ++k)
        for (long j = box[2]; j < box[3]; ++j)
            for (long i = box[0]; i < box[1]; ++i) sum += s->E[comp][o_idx(s, i, j, k)];
    return sum;
}

/* Transpose of one stretched B half update (sub-steps 1 and 5):
 *   psi' = b psi + c D_a E_c'   (only when advance)
 *   B_c -= dt/2 * sgn * (k D_a E_c' + psi')
 * for every face of component c and both curl terms.  aB is the adjoint of
 * B (unchanged), aE and apsi are updated in place. */
static void o_adj_half_B(oracle_sim *s, double **aE, double **aB, double *(*apsi)[3], int advance)
{
    double h = 0.5 * s->dt;
    for (int c = 0; c < 3; ++c) {
        int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
        /* (curl E)_c = D_{a1} E_{a2} - D_{a2} E_{a1} */
        int ax[2] = {a1, a2};
        int ec[2] = {a2, a1};
        double sg[2] = {1.0, -1.0};
        for (int t = 0; t < 2; ++t) {
            int a = ax[t];
            for (long k = 0; k < s->n[2]; ++k)
                for (long j = 0; j < s->n[1]; ++j)
                    for (long i = 0; i < s->n[0]; ++i) {
                        long ijk[3] = {i, j, k};
                        long e = o_idx(s, i, j, k);
                        long ia = ijk[a];
                        double coefB = -h * sg[t];         /* dB / d(stretched derivative) */
                        double w = coefB * s->kih[a][ia] * aB[c][e];
                        if (apsi[c][a]) {
                            double tot = apsi[c][a][e] + coefB * aB[c][e];
                            if (advance) {
                                w += s->ch[a][ia] * tot;
                                apsi[c][a][e] = s->bh[a][ia] * tot;
                            } else {
                                apsi[c][a][e] = tot;
                            }
                        }
                        /* D_a E at e: (E[p + e_a] - E[p]) / d_a; transpose scatters w/d */
                        long p[3] = {i, j, k};
                        p[a] += 1;
                        aE[ec[t]][o_idx(s, p[0], p[1], p[2])] += w / s->d[a];
                        aE[ec[t]][e] -= w / s->d[a];
                    }
        }
    }
}

/* The reverse sweep; when aE0, aB0, aJ0 are not NULL they receive the adjoint of the initial state
 * (dJ/dE^0, dJ/dB^0, dJ/dJs^0 at the state passed to the run, with the PML variables held fixed). */
static int o_adjoint(oracle_sim *s, long nsteps, int pid, double f0, double *grad_ell, double *grad_sig, double *out,
                     double *const *aE0, double *const *aB0, double *const *aJ0)
{
    const double twopi = 2.0 * 3.14159265358979323846;
    if (pid < 0 || pid >= s->nprobe || nsteps < 1) return -1;
    const o_probe *q = &s->probe[pid];
    long N = o_cells(s);
    double dt = s->dt, th = s->theta;

    /* forward, storing every state and the samples */
    o_state *traj = (o_state *)calloc((size_t)nsteps + 1, sizeof(o_state));
    double *samp = (double *)calloc((size_t)nsteps + 1, sizeof(double));
    double *Epre[3];
    for (long n = 0; n <= nsteps; ++n) o_state_alloc(s, &traj[n]);
    o_state_copy(s, &traj[0], s->E, s->B, s->J, s->psiB, s->psiE);
    long step0 = s->step;
    samp[0] = o_probe_sum(s, q->comp, q->box);
    for (long n = 0; n < nsteps; ++n) {
        oracle_step(s, 1);
        o_state_copy(s, &traj[n + 1], s->E, s->B, s->J, s->psiB, s->psiE);
        samp[n + 1] = o_probe_sum(s, q->comp, q->box);
    }
    double Fr = 0.0, Fi = 0.0;
    for (long n = 0; n <= nsteps; ++n) {
        double ph = twopi * f0 * (double)n * dt;
        Fr += samp[n] * dt * cos(ph);
        Fi -= samp[n] * dt * sin(ph);
    }

    /* adjoint state and per-edge gradients */
    double *aE[3], *aB[3], *aJ[3], *aH[3], *gl[3], *gs[3];
    double *apsiB[3][3], *apsiE[3][3];
    for (int c = 0; c < 3; ++c) {
        aE[c] = o_zeros(N); aB[c] = o_zeros(N); aJ[c] = o_zeros(N); aH[c] = o_zeros(N);
        gl[c] = o_zeros(N); gs[c] = o_zeros(N); Epre[c] = o_zeros(N);
        for (int a = 0; a < 3; ++a) {
            apsiB[c][a] = s->psiB[c][a] ? o_zeros(N) : NULL;
            apsiE[c][a] = s->psiE[c][a] ? o_zeros(N) : NULL;
        }
    }
    double *Hn[3];
    for (int c = 0; c < 3; ++c) Hn[c] = o_zeros(N);

    for (long n = nsteps; n >= 0; --n) {
        /* objective source at E^n: dJ/ds_n = 2 Re(conj(F) w_n) */
        double ph = twopi * f0 * (double)n * dt;
        double gn = 2.0 * dt * (Fr * cos(ph) - Fi * sin(ph));
        for (long k = q->box[4]; k < q->box[5]; ++k)
            for (long j = q->box[2]; j < q->box[3]; ++j)
                for (long i = q->box[0]; i < q->box[1]; ++i) aE[q->comp][o_idx(s, i, j, k)] += gn;
        if (n == 0) break;
        long m = n - 1; /* transpose step m -> m+1 */
        /* recompute the intermediates of step m: B^{m+1/2} (for H) and E^{m+1} before the sources */
        o_state_load(s, &traj[m]);
        s->step = step0 + m;
        o_half_B(s, 0);
        o_half_J(s);
        {
            int nsrc = s->nsrc;
            s->nsrc = 0;
            o_full_E(s);
            s->nsrc = nsrc;
        }
        for (int c = 0; c < 3; ++c) memcpy(Epre[c], s->E[c], (size_t)N * sizeof(double));
        const o_state *X0 = &traj[m], *X1 = &traj[m + 1];

        /* 5^T */
        o_adj_half_B(s, aE, aB, apsiB, 1);
        /* 4^T: Js^{m+1} = Js^{m+1/2} + dt/2 ell E^{m+1}/mu0 */
        for (int c = 0; c < 3; ++c)
            for (long e = 0; e < N; ++e)
                if (s->ell[c][e] > 0.0) {
                    aE[c][e] += 0.5 * dt * s->ell[c][e] / O_MU0 * aJ[c][e];
                    gl[c][e] += 0.5 * dt * X1->E[c][e] / O_MU0 * aJ[c][e];
                }
        /* 3^T: E^{m+1} = alpha [(1-(1-th) s) E^m + dt/eps (curlH - Js)], curlH from H = B^{m+1/2}/mu0 */
        for (int c = 0; c < 3; ++c) memset(aH[c], 0, (size_t)N * sizeof(double));
        for (int c = 0; c < 3; ++c) {
            int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
            int ax[2] = {a1, a2};
            int hc[2] = {a2, a1};
            double sg[2] = {1.0, -1.0};
            for (long k = 0; k < s->n[2]; ++k)
                for (long j = 0; j < s->n[1]; ++j)
                    for (long i = 0; i < s->n[0]; ++i) {
                        long ijk[3] = {i, j, k};
                        long e = o_idx(s, i, j, k);
                        if (o_on_wall(s, c, ijk)) aE[c][e] = 0.0;
                        double eps = s->eps[c][e];
                        double sgm = s->sig[c][e] * dt / eps;
                        double alpha = 1.0 / (1.0 + th * sgm);
                        double aEp = aE[c][e];
                        gs[c][e] += aEp * (dt / eps) * (-(1.0 - th) * X0->E[c][e] - th * Epre[c][e]) * alpha;
                        if (s->ell[c][e] > 0.0) aJ[c][e] -= alpha * (dt / eps) * aEp;
                        double cbar = alpha * (dt / eps) * aEp;
                        for (int t = 0; t < 2; ++t) {
                            int a = ax[t];
                            long ia = ijk[a];
                            double w = sg[t] * s->kin[a][ia] * cbar;
                            if (apsiE[c][a]) {
                                double tot = apsiE[c][a][e] + sg[t] * cbar;
                                w += s->cn[a][ia] * tot;
                                apsiE[c][a][e] = s->bn[a][ia] * tot;
                            }
                            /* D*_a H at e: (H[p] - H[p - e_a]) / d_a */
                            long p[3] = {i, j, k};
                            p[a] -= 1;
                            aH[hc[t]][e] += w / s->d[a];
                            aH[hc[t]][o_idx(s, p[0], p[1], p[2])] -= w / s->d[a];
                        }
                        aE[c][e] = alpha * (1.0 - (1.0 - th) * sgm) * aEp;
                    }
        }
        for (int c = 0; c < 3; ++c)
            for (long e = 0; e < N; ++e) aB[c][e] += aH[c][e] / O_MU0;
        /* 2^T: Js^{m+1/2} = Js^m + dt/2 ell E^m / mu0 */
        for (int c = 0; c < 3; ++c)
            for (long e = 0; e < N; ++e)
                if (s->ell[c][e] > 0.0) {
                    aE[c][e] += 0.5 * dt * s->ell[c][e] / O_MU0 * aJ[c][e];
                    gl[c][e] += 0.5 * dt * X0->E[c][e] / O_MU0 * aJ[c][e];
                }
        /* 1^T */
        o_adj_half_B(s, aE, aB, apsiB, 0);
    }
    if (aE0 && aB0 && aJ0)
        for (int c = 0; c < 3; ++c) {
            memcpy(aE0[c], aE[c], (size_t)N * sizeof(double));
            memcpy(aB0[c], aB[c], (size_t)N * sizeof(double));
            memcpy(aJ0[c], aJ[c], (size_t)N * sizeof(double));
        }
    /* restore the forward end state */
    o_state_load(s, &traj[nsteps]);
    s->step = step0 + nsteps;

    /* per-edge -> per-cell (the derivative of the edge material rule) */
    memset(grad_ell, 0, (size_t)N * sizeof(double));
    memset(grad_sig, 0, (size_t)N * sizeof(double));
    for (int c = 0; c < 3; ++c) {
        int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
        for (long k = 0; k < s->n[2]; ++k)
            for (long j = 0; j < s->n[1]; ++j)
                for (long i = 0; i < s->n[0]; ++i) {
                    long e = o_idx(s, i, j, k);
                    long cells[4];
                    int nsc = 0;
                    for (int u = 0; u < 2; ++u)
                        for (int v = 0; v < 2; ++v) {
                            long o[3] = {i, j, k};
                            o[a1] -= u;
                            o[a2] -= v;
                            cells[2 * u + v] = o_idx(s, o[0], o[1], o[2]);
                        }
                    (void)nsc;
                    double ls[4];
                    int cnt = 0;
                    const double *ellc = s->cell_ell;
                    for (int t = 0; t < 4; ++t) { ls[t] = ellc[cells[t]]; if (ls[t] > 0.0) cnt++; }
                    for (int t = 0; t < 4; ++t) {
                        if (cnt > 0) {
                            if (ls[t] > 0.0) {
                                grad_ell[cells[t]] += gl[c][e] / (double)cnt;
                                grad_sig[cells[t]] += gs[c][e] / (double)cnt;
                            }
                        } else {
                            grad_sig[cells[t]] += gs[c][e] / 4.0;
                        }
                    }
                }
    }
    if (out) { out[0] = Fr * Fr + Fi * Fi; out[1] = Fr; out[2] = Fi; }

    for (long n = 0; n <= nsteps; ++n) o_state_free(&traj[n]);
    free(traj); free(samp);
    for (int c = 0; c < 3; ++c) {
        free(aE[c]); free(aB[c]); free(aJ[c]); free(aH[c]); free(gl[c]); free(gs[c]); free(Epre[c]); free(Hn[c]);
        for (int a = 0; a < 3; ++a) { free(apsiB[c][a]); free(apsiE[c][a]); }
    }
    return 0;
}

int oracle_adjoint(oracle_sim *s, long nsteps, int pid, double f0, double *grad_ell, double *grad_sig, double *out)
{
    return o_adjoint(s, nsteps, pid, f0, grad_ell, grad_sig, out, NULL, NULL, NULL);
}

int oracle_adjoint_state(oracle_sim *s, long nsteps, int pid, double f0, double *grad_ell, double *grad_sig,
                         double *out, double *const *aE0, double *const *aB0, double *const *aJ0)
{
    return o_adjoint(s, nsteps, pid, f0, grad_ell, grad_sig, out, aE0, aB0, aJ0);
}
