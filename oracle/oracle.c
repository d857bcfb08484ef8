/*
 * Plain FP64 CPU oracle for the Downstream tracking + two-track vertexing
 * hot path (Kholoimov et al., "A Downstream and Vertexing Algorithm for Long
 * Lived Particles (LLP) Selection at the First High Level Trigger (HLT1) of
 * LHCb", arXiv:2503.13092).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * definition the GPU library is checked against.  It shares no code, header,
 * constant table or helper with the GPU library, and only the test suite,
 * the package smoke check and the benchmark's CPU-baseline leg may load it.
 * The product path never calls it.
 *
 * Everything is float64.  Inputs arrive as float64 arrays (callers convert
 * the float32 boundary values exactly).  Steps follow the paper's order:
 *
 *   O2  magnet-point (kink) extrapolation of a SciFi seed
 *       ("Algorithm Design", eq. 1 and the magnet-point text after it)
 *   O3  first search window in the last UT layer, UTbX (Dv0, same section)
 *   O4  refined windows through each UTbX hit and the magnet point
 *   O5  candidates: closest UTaX hit x 2 closest UTaU x 2 closest UTbV hits
 *       per UTbX hit, up to 10 UTbX hits; validity from the UT
 *       reconstructibility rule ("Track Types at LHCb")
 *   O6  least-squares x-z line fit and chi2 per candidate
 *   O7  one final candidate per SciFi seed (best score)
 *   O8  track state at the UT midpoint and q/p from the kink
 *   O9  ghost-killer feed-forward network and the "response < threshold"
 *       filter ("Ghost-Killer Neural Network", "Ghost Rejection")
 *   O3' Dv1 instead of O3 ("Algorithm Design", the improved version): no
 *       momentum window in UTbX; every UTbX hit in a Y sector compatible with
 *       the seed forms, with the magnet point, a line that must meet a UTaX
 *       hit (the axial triplet); stereo hits are added as in Dv0
 *   O10 two-track vertexing: trajectories of eq. 4 with gamma from eq. 3,
 *       Newton-Raphson point of closest approach, opposite charges, DOCA cut
 *       ("Vertexing Two Downstream Tracks", "Expected Physics Impact")
 *
 * Readings where the paper is silent (window sizes, the score being a
 * least-squares chi2, tie-breaks, the 17 ghost-killer features, the
 * straight-line Newton start, ...) are the documented readings of the
 * project; every one is listed in the design notes.
 *
 * Window and feature constants: parity unpinned against the paper (it prints
 * none); pinned only by the tests' closed-form, brute-force and library
 * comparisons.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    double z_layer[4];
    double tan_stereo[4];
    double z_magnet, z_seed, z_ref;
    double kick, polarity;
    double sigma_hit;
    double w1_c0, w1_c1, w2_c0, w2_c1;
    int max_l3;
    int n_closest[3];
    double gamma_c0, gamma_c1, fringe_polarity;
    int newton_iters;
    double doca_max;
    /* Dv1: algorithm 1 selects the triplet search; hits carry a Y sector
     * k = floor((y - sector_y0) / sector_h) in [0, n_sectors) */
    int algorithm;
    int n_sectors;
    double sector_y0, sector_h, sector_tol;
} orc_geom;

/* ---------------------------------------------------------------- O2 ---- */

/* Seed state s = (x, y, tx, ty, q/p) at z_seed.  The magnet point is the
 * straight-line extrapolation of the seed to z_magnet; before the kink the
 * slope is tx - MP*K*q/p; y is a straight line (the field is along y, so
 * there is no bending in y). */
void orc_extrapolate(const orc_geom *g, const double *s, double *x_before, double *y_at, double *x_magnet)
{
    double xm = s[0] + s[2] * (g->z_magnet - g->z_seed);
    double tb = s[2] - g->polarity * g->kick * s[4];
    for (int L = 0; L < 4; ++L) {
        x_before[L] = xm + tb * (g->z_layer[L] - g->z_magnet);
        y_at[L] = s[1] + s[3] * (g->z_layer[L] - g->z_seed);
    }
    *x_magnet = xm;
}

/* ----------------------------------------------------------- windows ---- */

typedef struct {
    int idx;       /* index within the (event, layer) run */
    double adelta; /* |x_hat - centre| */
    double u;
} win_hit;

static int cmp_win_hit(const void *pa, const void *pb)
{
    const win_hit *a = (const win_hit *)pa, *b = (const win_hit *)pb;
    if (a->adelta < b->adelta) return -1;
    if (a->adelta > b->adelta) return 1;
    if (a->u < b->u) return -1;
    if (a->u > b->u) return 1;
    return (a->idx > b->idx) - (a->idx < b->idx);
}

typedef struct {
    double edge_margin; /* smallest | |delta| - W | over hits looked at */
    double rank_gap;    /* smallest |delta| gap between last kept and first dropped */
} fragility;

/* All hits of one layer whose x_hat = u + y*tan(alpha) lies within W of the
 * centre (inclusive), ordered by (|delta|, u, index) and cut to `cap`.  A
 * full scan: no sorting of the hits, no binary search.  With `sec` given,
 * only hits whose Y sector lies in [klo, khi] are looked at. */
static int window(const double *u, const int *sec, int klo, int khi, int n, double y, double tana, double centre,
                  double W, int cap, win_hit *out, win_hit *scratch, fragility *fr)
{
    if (cap <= 0) return 0;
    int m = 0;
    for (int i = 0; i < n; ++i) {
        if (sec && (sec[i] < klo || sec[i] > khi)) continue;
        double xhat = u[i] + y * tana;
        double d = fabs(xhat - centre);
        double margin = fabs(d - W);
        if (margin < fr->edge_margin) fr->edge_margin = margin;
        if (d <= W) {
            scratch[m].idx = i;
            scratch[m].adelta = d;
            scratch[m].u = u[i];
            ++m;
        }
    }
    qsort(scratch, (size_t)m, sizeof(win_hit), cmp_win_hit);
    if (m > cap) {
        double gap = scratch[cap].adelta - scratch[cap - 1].adelta;
        if (gap < fr->rank_gap) fr->rank_gap = gap;
        m = cap;
    }
    memcpy(out, scratch, (size_t)m * sizeof(win_hit));
    return m;
}

/* ---------------------------------------------------------------- O6 ---- */

/* Weighted least-squares straight line x = a + b*(z - z_ref) through n points
 * with equal resolution sigma: closed-form 2x2 normal equations. */
void orc_fit(int n, const double *dz, const double *x, double sigma, double *a, double *b, double *chi2)
{
    double w = 1.0 / (sigma * sigma);
    double S = 0, Sz = 0, Szz = 0, Sx = 0, Szx = 0;
    for (int i = 0; i < n; ++i) {
        S += w;
        Sz += w * dz[i];
        Szz += w * dz[i] * dz[i];
        Sx += w * x[i];
        Szx += w * dz[i] * x[i];
    }
    double det = S * Szz - Sz * Sz;
    double bb = (S * Szx - Sz * Sx) / det;
    double aa = (Szz * Sx - Sz * Szx) / det;
    double c2 = 0;
    for (int i = 0; i < n; ++i) {
        double r = x[i] - aa - bb * dz[i];
        c2 += w * r * r;
    }
    *a = aa;
    *b = bb;
    *chi2 = c2;
}

/* ------------------------------------------------------------ O3..O8 ---- */

typedef struct {
    int c;          /* candidate index (mixed radix over the rank lists) */
    int hit[4];     /* index within the layer run, -1 = none */
    int nhits;
    int valid;
    double a, b, chi2;
} cand_t;

/* Enumerate every candidate of one seed in rank order (O3-O6).  `u[L]` is the
 * hit run of layer L (n[L] hits).  Returns the number of candidates written
 * (at most max_out), and the number that would have been written in *total. */
static int enumerate_dv1(const orc_geom *g, const double *s, const double *const *u, const int *const *sec,
                         const int *n, cand_t *out, int max_out, int *total, fragility *fr, win_hit *scratch);

static int enumerate_candidates(const orc_geom *g, const double *s, const double *const *u,
                                const int *const *sec, const int *n, cand_t *out, int max_out, int *total,
                                fragility *fr, win_hit *scratch)
{
    if (g->algorithm == 1) return enumerate_dv1(g, s, u, sec, n, out, max_out, total, fr, scratch);
    double xb[4], yL[4], xm;
    orc_extrapolate(g, s, xb, yL, &xm);
    double aq = fabs(s[4]);
    double W1 = g->w1_c0 + g->w1_c1 * aq;
    double W2 = g->w2_c0 + g->w2_c1 * aq;
    int cap3 = g->max_l3;
    win_hit *A3 = (win_hit *)malloc(sizeof(win_hit) * (size_t)(cap3 > 0 ? cap3 : 1));
    int n3 = window(u[3], NULL, 0, 0, n[3], yL[3], g->tan_stereo[3], xb[3], W1, cap3, A3, scratch, fr);
    int nw[3];
    for (int L = 0; L < 3; ++L) nw[L] = g->n_closest[L] > 0 ? g->n_closest[L] : 1;
    int cnt = 0;
    win_hit AL[3][64];
    for (int r3 = 0; r3 < n3; ++r3) {
        double xh3 = u[3][A3[r3].idx] + yL[3] * g->tan_stereo[3];
        double tprime = (xm - xh3) / (g->z_magnet - g->z_layer[3]);
        int nA[3];
        for (int L = 0; L < 3; ++L) {
            double xr = xh3 + tprime * (g->z_layer[L] - g->z_layer[3]);
            int cap = g->n_closest[L] < 64 ? g->n_closest[L] : 64;
            nA[L] = window(u[L], NULL, 0, 0, n[L], yL[L], g->tan_stereo[L], xr, W2, cap, AL[L], scratch, fr);
        }
        /* option lists: the ranked window hits, or {none} if the window is empty */
        int no[3];
        for (int L = 0; L < 3; ++L) no[L] = nA[L] > 0 ? nA[L] : 1;
        for (int i0 = 0; i0 < no[0]; ++i0)
            for (int i1 = 0; i1 < no[1]; ++i1)
                for (int i2 = 0; i2 < no[2]; ++i2) {
                    cand_t cd;
                    cd.c = ((r3 * nw[0] + i0) * nw[1] + i1) * nw[2] + i2;
                    cd.hit[3] = A3[r3].idx;
                    cd.hit[0] = nA[0] > 0 ? AL[0][i0].idx : -1;
                    cd.hit[1] = nA[1] > 0 ? AL[1][i1].idx : -1;
                    cd.hit[2] = nA[2] > 0 ? AL[2][i2].idx : -1;
                    double dz[4], xx[4];
                    int k = 0;
                    for (int L = 0; L < 4; ++L) {
                        if (cd.hit[L] < 0) continue;
                        dz[k] = g->z_layer[L] - g->z_ref;
                        xx[k] = u[L][cd.hit[L]] + yL[L] * g->tan_stereo[L];
                        ++k;
                    }
                    cd.nhits = k;
                    /* UT rule: >= 3 hits here, one of them in UTaX or UTaU; UTbX is always present */
                    cd.valid = (k >= 3) && (cd.hit[0] >= 0 || cd.hit[1] >= 0);
                    cd.a = cd.b = cd.chi2 = 0.0;
                    if (k >= 2) orc_fit(k, dz, xx, g->sigma_hit, &cd.a, &cd.b, &cd.chi2);
                    if (cnt < max_out) out[cnt] = cd;
                    ++cnt;
                }
    }
    free(A3);
    *total = cnt;
    return cnt < max_out ? cnt : max_out;
}

/* Y sectors compatible with height y: the sectors k whose band
 * [y0 + k h, y0 + (k + 1) h) overlaps [y - tol, y + tol] (y is a straight
 * line: no field component bends it); klo > khi when none does.  The
 * distance of y -/+ tol to the nearest sector boundary goes to the edge
 * margin. */
static void sector_range(const orc_geom *g, double y, int *klo, int *khi, fragility *fr)
{
    double a = (y - g->sector_tol - g->sector_y0) / g->sector_h;
    double b = (y + g->sector_tol - g->sector_y0) / g->sector_h;
    double ma = fabs(a - floor(a + 0.5)) * g->sector_h, mb = fabs(b - floor(b + 0.5)) * g->sector_h;
    if (ma < fr->edge_margin) fr->edge_margin = ma;
    if (mb < fr->edge_margin) fr->edge_margin = mb;
    double fa = floor(a), fb = floor(b);
    double top = (double)(g->n_sectors - 1);
    /* outside every band: an empty range */
    if (fb < 0.0 || fa > top) {
        *klo = 1;
        *khi = 0;
        return;
    }
    *klo = (int)(fa < 0.0 ? 0.0 : fa);
    *khi = (int)(fb > top ? top : fb);
}

/* Dv1 (O3'): candidates of one seed from axial triplets.  Every UTbX hit of
 * a compatible Y sector, in index order (no momentum window), defines with
 * the magnet point a straight line; the line's refined windows in UTaX, UTaU
 * and UTbV are those of Dv0 restricted to compatible sectors.  A triplet
 * needs a UTaX hit; the stereo options and the fit follow Dv0.  Candidate
 * index: ((i3 * nw0 + i0) * nw1 + i1) * nw2 + i2, i3 the UTbX hit's index in
 * its layer run.  With sec == NULL every hit counts as compatible. */
static int enumerate_dv1(const orc_geom *g, const double *s, const double *const *u, const int *const *sec,
                         const int *n, cand_t *out, int max_out, int *total, fragility *fr, win_hit *scratch)
{
    double xb[4], yL[4], xm;
    orc_extrapolate(g, s, xb, yL, &xm);
    double W2 = g->w2_c0 + g->w2_c1 * fabs(s[4]);
    int klo[4] = {0, 0, 0, 0}, khi[4] = {0, 0, 0, 0};
    for (int L = 0; L < 4; ++L)
        if (sec) sector_range(g, yL[L], &klo[L], &khi[L], fr);
    int nw[3];
    for (int L = 0; L < 3; ++L) nw[L] = g->n_closest[L] > 0 ? g->n_closest[L] : 1;
    int cnt = 0;
    win_hit AL[3][64];
    for (int i3 = 0; i3 < n[3]; ++i3) {
        if (sec && (sec[3][i3] < klo[3] || sec[3][i3] > khi[3])) continue;
        double xh3 = u[3][i3] + yL[3] * g->tan_stereo[3];
        double tprime = (xm - xh3) / (g->z_magnet - g->z_layer[3]);
        int nA[3];
        for (int L = 0; L < 3; ++L) {
            double xr = xh3 + tprime * (g->z_layer[L] - g->z_layer[3]);
            int cap = g->n_closest[L] < 64 ? g->n_closest[L] : 64;
            nA[L] = window(u[L], sec ? sec[L] : NULL, klo[L], khi[L], n[L], yL[L], g->tan_stereo[L], xr, W2, cap,
                           AL[L], scratch, fr);
        }
        if (nA[0] == 0) continue; /* no axial triplet */
        int no[3];
        for (int L = 0; L < 3; ++L) no[L] = nA[L] > 0 ? nA[L] : 1;
        for (int i0 = 0; i0 < no[0]; ++i0)
            for (int i1 = 0; i1 < no[1]; ++i1)
                for (int i2 = 0; i2 < no[2]; ++i2) {
                    cand_t cd;
                    cd.c = ((i3 * nw[0] + i0) * nw[1] + i1) * nw[2] + i2;
                    cd.hit[3] = i3;
                    cd.hit[0] = AL[0][i0].idx;
                    cd.hit[1] = nA[1] > 0 ? AL[1][i1].idx : -1;
                    cd.hit[2] = nA[2] > 0 ? AL[2][i2].idx : -1;
                    double dz[4], xx[4];
                    int k = 0;
                    for (int L = 0; L < 4; ++L) {
                        if (cd.hit[L] < 0) continue;
                        dz[k] = g->z_layer[L] - g->z_ref;
                        xx[k] = u[L][cd.hit[L]] + yL[L] * g->tan_stereo[L];
                        ++k;
                    }
                    cd.nhits = k;
                    cd.valid = k >= 3; /* UTaX is present in every triplet */
                    cd.a = cd.b = cd.chi2 = 0.0;
                    orc_fit(k, dz, xx, g->sigma_hit, &cd.a, &cd.b, &cd.chi2);
                    if (cnt < max_out) out[cnt] = cd;
                    ++cnt;
                }
    }
    *total = cnt;
    return cnt < max_out ? cnt : max_out;
}

/* lexicographic (more hits, lower chi2, lower candidate index) */
static int better(const cand_t *x, const cand_t *y)
{
    if (x->nhits != y->nhits) return x->nhits > y->nhits;
    if (x->chi2 != y->chi2) return x->chi2 < y->chi2;
    return x->c < y->c;
}

/* Candidate list of one seed, for brute-force comparisons in the tests. */
int orc_candidates(const orc_geom *g, const double *s, const double *u0, int n0, const double *u1, int n1,
                   const double *u2, int n2, const double *u3, int n3, const int *sec0, const int *sec1,
                   const int *sec2, const int *sec3, int max_out, int *c_out, int *hits_out, int *nhits_out,
                   int *valid_out, double *a_out, double *b_out, double *chi2_out)
{
    const double *u[4] = {u0, u1, u2, u3};
    const int *sec[4] = {sec0, sec1, sec2, sec3};
    int n[4] = {n0, n1, n2, n3};
    int big = n0 + n1 + n2 + n3 + 1;
    win_hit *scratch = (win_hit *)malloc(sizeof(win_hit) * (size_t)big);
    cand_t *cands = (cand_t *)malloc(sizeof(cand_t) * (size_t)(max_out > 0 ? max_out : 1));
    fragility fr = {INFINITY, INFINITY};
    int total = 0;
    int m = enumerate_candidates(g, s, u, sec0 ? sec : NULL, n, cands, max_out, &total, &fr, scratch);
    for (int i = 0; i < m; ++i) {
        c_out[i] = cands[i].c;
        for (int L = 0; L < 4; ++L) hits_out[4 * i + L] = cands[i].hit[L];
        nhits_out[i] = cands[i].nhits;
        valid_out[i] = cands[i].valid;
        a_out[i] = cands[i].a;
        b_out[i] = cands[i].b;
        chi2_out[i] = cands[i].chi2;
    }
    free(scratch);
    free(cands);
    return total;
}

typedef struct {
    const orc_geom *g;
    int e_begin, e_end;
    const int *seed_off;
    const double *sx, *sy, *stx, *sty, *sqop;
    const int *hit_off;
    const double *hu;
    const int *hsec; /* Y sector per hit (Dv1), may be NULL */
    /* outputs per seed */
    double *x, *y, *tx, *ty, *qop, *chi2;
    int *nhits, *hits, *cand;
    double *edge_margin, *chi2_gap, *rank_gap;
} track_job;

static int all_finite(const double *v, int n)
{
    for (int i = 0; i < n; ++i)
        if (!isfinite(v[i])) return 0;
    return 1;
}

static void empty_track(track_job *J, int i)
{
    J->x[i] = J->y[i] = J->tx[i] = J->ty[i] = J->qop[i] = J->chi2[i] = 0.0;
    J->nhits[i] = 0;
    J->cand[i] = -1;
    for (int L = 0; L < 4; ++L) J->hits[4 * i + L] = -1;
    J->edge_margin[i] = INFINITY;
    J->chi2_gap[i] = INFINITY;
    J->rank_gap[i] = INFINITY;
}

static void *track_worker(void *arg)
{
    track_job *J = (track_job *)arg;
    const orc_geom *g = J->g;
    int maxc = 1;
    {
        int per3 = 1;
        for (int L = 0; L < 3; ++L) per3 *= (g->n_closest[L] > 0 ? g->n_closest[L] : 1);
        maxc = (g->max_l3 > 0 ? g->max_l3 : 1) * per3;
    }
    int per3 = maxc / (g->max_l3 > 0 ? g->max_l3 : 1);
    cand_t *cands = (cand_t *)malloc(sizeof(cand_t) * (size_t)maxc);
    size_t scratch_n = 16;
    win_hit *scratch = (win_hit *)malloc(sizeof(win_hit) * scratch_n);
    for (int e = J->e_begin; e < J->e_end; ++e) {
        int s0 = J->seed_off[e], s1 = J->seed_off[e + 1];
        const double *u[4];
        const int *sec[4] = {NULL, NULL, NULL, NULL};
        int n[4];
        int tot = 0;
        for (int L = 0; L < 4; ++L) {
            u[L] = J->hu + J->hit_off[4 * e + L];
            if (J->hsec) sec[L] = J->hsec + J->hit_off[4 * e + L];
            n[L] = J->hit_off[4 * e + L + 1] - J->hit_off[4 * e + L];
            tot += n[L];
        }
        if (g->algorithm == 1 && n[3] * per3 > maxc) { /* Dv1: every UTbX hit may open candidates */
            maxc = n[3] * per3;
            cands = (cand_t *)realloc(cands, sizeof(cand_t) * (size_t)maxc);
        }
        if ((size_t)tot + 1 > scratch_n) {
            scratch_n = (size_t)tot + 1;
            scratch = (win_hit *)realloc(scratch, sizeof(win_hit) * scratch_n);
        }
        /* an event with a non-finite hit produces no tracks */
        int event_ok = all_finite(J->hu + J->hit_off[4 * e], tot);
        for (int i = s0; i < s1; ++i) {
            double s[5] = {J->sx[i], J->sy[i], J->stx[i], J->sty[i], J->sqop[i]};
            empty_track(J, i);
            if (!event_ok || !all_finite(s, 5)) continue;
            fragility fr = {INFINITY, INFINITY};
            int total = 0;
            int m = enumerate_candidates(g, s, u, J->hsec ? sec : NULL, n, cands, maxc, &total, &fr, scratch);
            int best = -1;
            for (int k = 0; k < m; ++k) {
                if (!cands[k].valid) continue;
                if (best < 0 || better(&cands[k], &cands[best])) best = k;
            }
            J->edge_margin[i] = fr.edge_margin;
            J->rank_gap[i] = fr.rank_gap;
            if (best < 0) continue;
            const cand_t *B = &cands[best];
            /* nearest competitor with the same number of hits */
            double gap = INFINITY;
            for (int k = 0; k < m; ++k) {
                if (k == best || !cands[k].valid || cands[k].nhits != B->nhits) continue;
                double d = fabs(cands[k].chi2 - B->chi2);
                if (d < gap) gap = d;
            }
            J->chi2_gap[i] = gap;
            J->x[i] = B->a;
            J->tx[i] = B->b;
            J->y[i] = s[1] + s[3] * (g->z_ref - g->z_seed);
            J->ty[i] = s[3];
            double mk = g->polarity * g->kick;
            J->qop[i] = (mk != 0.0) ? (s[2] - B->b) / mk : s[4];
            J->chi2[i] = B->chi2;
            J->nhits[i] = B->nhits;
            J->cand[i] = B->c;
            for (int L = 0; L < 4; ++L) J->hits[4 * i + L] = B->hit[L];
        }
    }
    free(cands);
    free(scratch);
    return NULL;
}

/* Tracks for every seed of a batch.  hits[4*i+L] is the selected hit's index
 * within the (event, layer L) run, -1 if none; nhits 0 = no track.
 * Diagnostics: edge_margin (distance of the closest looked-at hit to a window
 * edge), chi2_gap (chi2 distance to the nearest competing candidate with the
 * same number of hits), rank_gap (|delta| gap at a rank cut). */
int orc_find_tracks(const orc_geom *g, int n_events, const int *seed_off, const double *sx, const double *sy,
                    const double *stx, const double *sty, const double *sqop, const int *hit_off, const double *hu,
                    const int *hit_sector, double *x, double *y, double *tx, double *ty, double *qop, double *chi2, int *nhits, int *hits,
                    int *cand, double *edge_margin, double *chi2_gap, double *rank_gap, int n_threads)
{
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 256) n_threads = 256;
    if (n_threads > n_events) n_threads = n_events > 0 ? n_events : 1;
    pthread_t th[256];
    track_job jobs[256];
    for (int t = 0; t < n_threads; ++t) {
        track_job J = {g, (int)((long)n_events * t / n_threads), (int)((long)n_events * (t + 1) / n_threads),
                       seed_off, sx, sy, stx, sty, sqop, hit_off, hu, hit_sector, x, y, tx, ty, qop, chi2, nhits,
                       hits, cand,
                       edge_margin, chi2_gap, rank_gap};
        jobs[t] = J;
    }
    if (n_threads == 1) {
        track_worker(&jobs[0]);
        return 0;
    }
    for (int t = 0; t < n_threads; ++t) pthread_create(&th[t], NULL, track_worker, &jobs[t]);
    for (int t = 0; t < n_threads; ++t) pthread_join(th[t], NULL);
    return 0;
}

/* ------------------------------------------------------- clone killing ---- */

/* Clone killing ("Algorithm Design"): among found tracks of one event, a
 * track is killed when another track shares more than two of its UT hits
 * (same hit in the same layer) and has the better score.  Score order: more
 * hits, then lower chi2, then lower seed slot.  Every pair is compared on
 * the tracks as selected (a killed track still kills the tracks it beats).
 * Writes killed[i] = 1/0; chi2 is the stored (float32) value. */
int orc_kill_clones(int n_events, const int *seed_off, const int *nhits, const int *hits, const double *chi2,
                    int *killed)
{
    for (int e = 0; e < n_events; ++e) {
        int s0 = seed_off[e], s1 = seed_off[e + 1];
        for (int i = s0; i < s1; ++i) {
            killed[i] = 0;
            if (nhits[i] <= 0) continue;
            for (int j = s0; j < s1; ++j) {
                if (j == i || nhits[j] <= 0) continue;
                int shared = 0;
                for (int L = 0; L < 4; ++L)
                    if (hits[4 * i + L] >= 0 && hits[4 * i + L] == hits[4 * j + L]) ++shared;
                if (shared <= 2) continue;
                int j_better = nhits[j] > nhits[i] || (nhits[j] == nhits[i] && chi2[j] < chi2[i]) ||
                               (nhits[j] == nhits[i] && chi2[j] == chi2[i] && j < i);
                if (j_better) {
                    killed[i] = 1;
                    break;
                }
            }
        }
    }
    return 0;
}

/* ---------------------------------------------------------------- O9 ---- */

void orc_features(const orc_geom *g, const double *trk, int nh, const double *s, const double *hit_u, double *f);
double orc_mlp(const double *w, const double *f);

#define NF 17
#define NH1 32
#define NH2 16

/* Ghost-killer inputs of one stored track (state at z_ref, chi2, hit count),
 * its seed and its hits' u (NaN when the layer has no hit). */
void orc_features(const orc_geom *g, const double *trk /* x y tx ty qop chi2 */, int nh, const double *s,
                  const double *hit_u /* [4] */, double *f)
{
    double x = trk[0], y = trk[1], tx = trk[2], ty = trk[3];
    f[0] = x / 1000.0;
    f[1] = y / 1000.0;
    f[2] = tx / 0.3;
    f[3] = ty / 0.3;
    f[4] = trk[4] / 0.5;
    f[5] = trk[5] / 10.0;
    f[6] = (nh - 3.5) / 0.5;
    f[7] = s[0] / 3000.0;
    f[8] = s[1] / 3000.0;
    f[9] = s[2] / 0.5;
    f[10] = s[3] / 0.5;
    f[11] = s[4] / 0.5;
    for (int L = 0; L < 4; ++L) {
        if (isnan(hit_u[L])) {
            f[12 + L] = 0.0;
            continue;
        }
        double dz = g->z_layer[L] - g->z_ref;
        double yl = y + ty * dz;
        double xhat = hit_u[L] + yl * g->tan_stereo[L];
        double r = xhat - (x + tx * dz);
        f[12 + L] = r / g->sigma_hit / 5.0;
    }
    double x_at_magnet = x + tx * (g->z_magnet - g->z_ref);
    double xm_seed = s[0] + s[2] * (g->z_magnet - g->z_seed);
    f[16] = x_at_magnet - xm_seed;
}

/* 17 -> 32 ReLU -> 16 ReLU -> 1 sigmoid; w = W1[32][17] b1 W2[16][32] b2 W3[1][16] b3 */
double orc_mlp(const double *w, const double *f)
{
    const double *W1 = w, *b1 = W1 + NH1 * NF, *W2 = b1 + NH1, *b2 = W2 + NH2 * NH1, *W3 = b2 + NH2,
                 *b3 = W3 + NH2;
    double h1[NH1], h2[NH2];
    for (int j = 0; j < NH1; ++j) {
        double a = b1[j];
        for (int k = 0; k < NF; ++k) a += W1[j * NF + k] * f[k];
        h1[j] = a > 0.0 ? a : 0.0;
    }
    for (int j = 0; j < NH2; ++j) {
        double a = b2[j];
        for (int k = 0; k < NH1; ++k) a += W2[j * NH1 + k] * h1[k];
        h2[j] = a > 0.0 ? a : 0.0;
    }
    double z = b3[0];
    for (int k = 0; k < NH2; ++k) z += W3[k] * h2[k];
    return 1.0 / (1.0 + exp(-z));
}

/* Score every found track of a batch (score = 0 for seeds without a track).
 * Track values are the stored float32 values, passed as float64. */
int orc_ghost_kill(const orc_geom *g, int n_events, const int *seed_off, const double *sx, const double *sy,
                   const double *stx, const double *sty, const double *sqop, const int *hit_off, const double *hu,
                   const double *x, const double *y, const double *tx, const double *ty, const double *qop,
                   const double *chi2, const int *nhits, const int *hits, const double *w, double *score,
                   double *features /* nullable, [S*17] */)
{
    for (int e = 0; e < n_events; ++e) {
        for (int i = seed_off[e]; i < seed_off[e + 1]; ++i) {
            score[i] = 0.0;
            if (features)
                for (int k = 0; k < NF; ++k) features[(size_t)i * NF + k] = 0.0;
            if (nhits[i] <= 0) continue;
            double trk[6] = {x[i], y[i], tx[i], ty[i], qop[i], chi2[i]};
            double s[5] = {sx[i], sy[i], stx[i], sty[i], sqop[i]};
            double hu4[4];
            for (int L = 0; L < 4; ++L) {
                int h = hits[4 * i + L];
                hu4[L] = h >= 0 ? hu[hit_off[4 * e + L] + h] : NAN;
            }
            double f[NF];
            orc_features(g, trk, nhits[i], s, hu4, f);
            if (features)
                for (int k = 0; k < NF; ++k) features[(size_t)i * NF + k] = f[k];
            score[i] = orc_mlp(w, f);
        }
    }
    return 0;
}

/* ------------------------------------------------ every candidate scored -- */

/* Every valid candidate of every seed as a track of its own ("Ghost-Killer
 * Neural Network": the network is trained on the candidates found with wide
 * windows and clone killing off): the candidate's fit stored as float32 like a
 * selected track, its 17 features and its score.  Rows are written in (seed,
 * candidate index) order; returns the number of rows (at most max_rows). */
int orc_score_candidates(const orc_geom *g, int n_events, const int *seed_off, const double *sx, const double *sy,
                         const double *stx, const double *sty, const double *sqop, const int *hit_off,
                         const double *hu, const double *w, int max_rows, int *row_seed, int *row_cand,
                         int *row_hits, int *row_nhits, double *row_state /* [6]: x y tx ty qop chi2 (f32) */,
                         double *row_score)
{
    /* candidate rows follow Dv0's enumeration */
    orc_geom g0 = *g;
    g0.algorithm = 0;
    g = &g0;
    int per3 = 1;
    for (int L = 0; L < 3; ++L) per3 *= (g->n_closest[L] > 0 ? g->n_closest[L] : 1);
    int maxc = (g->max_l3 > 0 ? g->max_l3 : 1) * per3;
    cand_t *cands = (cand_t *)malloc(sizeof(cand_t) * (size_t)maxc);
    int rows = 0;
    for (int e = 0; e < n_events; ++e) {
        const double *u[4];
        int n[4], tot = 0;
        for (int L = 0; L < 4; ++L) {
            u[L] = hu + hit_off[4 * e + L];
            n[L] = hit_off[4 * e + L + 1] - hit_off[4 * e + L];
            tot += n[L];
        }
        if (!all_finite(hu + hit_off[4 * e], tot)) continue;
        win_hit *scratch = (win_hit *)malloc(sizeof(win_hit) * (size_t)(tot + 1));
        for (int i = seed_off[e]; i < seed_off[e + 1]; ++i) {
            double s[5] = {sx[i], sy[i], stx[i], sty[i], sqop[i]};
            if (!all_finite(s, 5)) continue;
            fragility fr = {INFINITY, INFINITY};
            int total = 0;
            int m = enumerate_candidates(g, s, u, NULL, n, cands, maxc, &total, &fr, scratch);
            for (int k = 0; k < m; ++k) {
                const cand_t *cd = &cands[k];
                if (!cd->valid) continue;
                if (rows < max_rows) {
                    double mk = g->polarity * g->kick;
                    /* the stored float32 record, then features of it */
                    double trk[6];
                    trk[0] = (float)cd->a;
                    trk[1] = (float)(s[1] + s[3] * (g->z_ref - g->z_seed));
                    trk[2] = (float)cd->b;
                    trk[3] = (float)s[3];
                    trk[4] = (float)((mk != 0.0) ? (s[2] - cd->b) / mk : s[4]);
                    trk[5] = (float)cd->chi2;
                    double sf[5];
                    for (int q = 0; q < 5; ++q) sf[q] = (float)s[q];
                    double hu4[4];
                    for (int L = 0; L < 4; ++L) hu4[L] = cd->hit[L] >= 0 ? u[L][cd->hit[L]] : NAN;
                    double f[NF];
                    orc_features(g, trk, cd->nhits, sf, hu4, f);
                    row_seed[rows] = i;
                    row_cand[rows] = cd->c;
                    for (int L = 0; L < 4; ++L) row_hits[4 * rows + L] = cd->hit[L];
                    row_nhits[rows] = cd->nhits;
                    for (int q = 0; q < 6; ++q) row_state[6 * rows + q] = trk[q];
                    row_score[rows] = orc_mlp(w, f);
                }
                ++rows;
            }
        }
        free(scratch);
    }
    free(cands);
    return rows < max_rows ? rows : max_rows;
}

/* --------------------------------------------------------------- O10 ---- */

static void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Point of closest approach of two tracks (x, y, tx, ty, qop at z_ref).
 * Trajectory of eq. 4: x = x0 + tx*dz + gamma*dz^2, y = y0 + ty*dz, with
 * gamma(q/p) of eq. 3 (q/p in MeV^-1).  Start from the straight-line PCA,
 * then exactly `iters` Newton-Raphson steps on |T1(z1) - T2(z2)|^2.
 * Returns 1 and writes (vx, vy, vz, doca, z1, z2) on success, 0 if the pair
 * is (near-)parallel or the Newton system is singular. */
int orc_pca(const orc_geom *g, const double *t1, const double *t2, int iters, double *out)
{
    double fp = g->fringe_polarity;
    double gam1 = -fp * (g->gamma_c0 + g->gamma_c1 * (t1[4] * 1e-3));
    double gam2 = -fp * (g->gamma_c0 + g->gamma_c1 * (t2[4] * 1e-3));
    double d1[3] = {t1[2], t1[3], 1.0}, d2[3] = {t2[2], t2[3], 1.0};
    double w[3] = {t1[0] - t2[0], t1[1] - t2[1], 0.0};
    double nrm[3];
    cross3(d1, d2, nrm);
    double nn = dot3(nrm, nrm);
    if (nn < 1e-12) return 0;
    double wd[3];
    cross3(w, d2, wd);
    double s = -dot3(wd, nrm) / nn;
    cross3(w, d1, wd);
    double t = -dot3(wd, nrm) / nn;
    double z1 = g->z_ref + s, z2 = g->z_ref + t;
    for (int it = 0; it < iters; ++it) {
        double a1 = z1 - g->z_ref, a2 = z2 - g->z_ref;
        double T1[3] = {t1[0] + t1[2] * a1 + gam1 * a1 * a1, t1[1] + t1[3] * a1, z1};
        double T2[3] = {t2[0] + t2[2] * a2 + gam2 * a2 * a2, t2[1] + t2[3] * a2, z2};
        double P1[3] = {t1[2] + 2.0 * gam1 * a1, t1[3], 1.0};
        double P2[3] = {t2[2] + 2.0 * gam2 * a2, t2[3], 1.0};
        double D[3] = {T1[0] - T2[0], T1[1] - T2[1], T1[2] - T2[2]};
        double g1 = dot3(D, P1), g2 = -dot3(D, P2);
        double h11 = dot3(P1, P1) + D[0] * 2.0 * gam1;
        double h22 = dot3(P2, P2) - D[0] * 2.0 * gam2;
        double h12 = -dot3(P1, P2);
        double det = h11 * h22 - h12 * h12;
        double tr = h11 + h22;
        if (fabs(det) < 1e-12 * tr * tr) return 0;
        double dz1 = (h22 * g1 - h12 * g2) / det;
        double dz2 = (h11 * g2 - h12 * g1) / det;
        z1 -= dz1;
        z2 -= dz2;
    }
    double a1 = z1 - g->z_ref, a2 = z2 - g->z_ref;
    double T1[3] = {t1[0] + t1[2] * a1 + gam1 * a1 * a1, t1[1] + t1[3] * a1, z1};
    double T2[3] = {t2[0] + t2[2] * a2 + gam2 * a2 * a2, t2[1] + t2[3] * a2, z2};
    double D[3] = {T1[0] - T2[0], T1[1] - T2[1], T1[2] - T2[2]};
    out[0] = 0.5 * (T1[0] + T2[0]);
    out[1] = 0.5 * (T1[1] + T2[1]);
    out[2] = 0.5 * (T1[2] + T2[2]);
    out[3] = sqrt(dot3(D, D));
    out[4] = z1;
    out[5] = z2;
    return 1;
}

/* ---------------------------------------------- mass and trigger lines ---- */

#define LINE_NF 12
#define LINE_NH 32
#define LINE_NW (LINE_NH * LINE_NF + LINE_NH + LINE_NH + 1) /* 449 per line network */

/* After vertexing ("Vertexing Two Downstream Tracks"; mass after the vertex
 * correction, Fig. 18; "Expected Physics Impact": four one-hidden-layer
 * networks of 32 nodes over the two tracks and the vertex).  Momenta: |p| =
 * 1/|q/p| of each track's seed, direction = trajectory tangent at its point of
 * closest approach (z1, z2).  Masses in MeV: K0S hypothesis pi+ pi-, Lambda
 * hypothesis p pi with the proton the higher-momentum track.  Line inputs
 * (reading; the paper does not list them): ln p1, ln p2 (GeV), the four
 * tangent slopes, vertex z/1000, transverse radius/100, DOCA, (m_pipi -
 * 497.6)/100, (m_ppi - 1115.7)/100, pair pT (GeV).  out = m_pipi, m_ppi, s0..s3. */
void orc_vertex_extras(const orc_geom *g, const double *t1, const double *t2, double q1, double q2, double z1,
                       double z2, const double *vtx /* x y z doca */, const double *wl, double *out)
{
    const double MPI = 0.13957039, MP = 0.93827209;
    double fp = g->fringe_polarity;
    double gam1 = -fp * (g->gamma_c0 + g->gamma_c1 * (t1[4] * 1e-3));
    double gam2 = -fp * (g->gamma_c0 + g->gamma_c1 * (t2[4] * 1e-3));
    double a1 = z1 - g->z_ref, a2 = z2 - g->z_ref;
    double d1[3] = {t1[2] + 2.0 * gam1 * a1, t1[3], 1.0}, d2[3] = {t2[2] + 2.0 * gam2 * a2, t2[3], 1.0};
    double n1 = sqrt(dot3(d1, d1)), n2 = sqrt(dot3(d2, d2));
    double p1 = 1.0 / fabs(q1), p2 = 1.0 / fabs(q2);
    double P1[3], P2[3], S[3];
    for (int k = 0; k < 3; ++k) {
        P1[k] = p1 * d1[k] / n1;
        P2[k] = p2 * d2[k] / n2;
        S[k] = P1[k] + P2[k];
    }
    double ss = dot3(S, S);
    double e1 = sqrt(p1 * p1 + MPI * MPI), e2 = sqrt(p2 * p2 + MPI * MPI);
    double m2 = (e1 + e2) * (e1 + e2) - ss;
    out[0] = 1000.0 * sqrt(m2 > 0.0 ? m2 : 0.0);
    double ep = p1 >= p2 ? sqrt(p1 * p1 + MP * MP) + e2 : sqrt(p2 * p2 + MP * MP) + e1;
    m2 = ep * ep - ss;
    out[1] = 1000.0 * sqrt(m2 > 0.0 ? m2 : 0.0);
    double f[LINE_NF] = {log(p1), log(p2), d1[0] / 0.3, d1[1] / 0.3, d2[0] / 0.3, d2[1] / 0.3, vtx[2] / 1000.0,
                         sqrt(vtx[0] * vtx[0] + vtx[1] * vtx[1]) / 100.0, vtx[3], (out[0] - 497.6) / 100.0,
                         (out[1] - 1115.7) / 100.0, sqrt(S[0] * S[0] + S[1] * S[1])};
    for (int l = 0; l < 4; ++l) {
        const double *W = wl + (size_t)l * LINE_NW, *b1 = W + LINE_NH * LINE_NF, *w2 = b1 + LINE_NH,
                     *b2 = w2 + LINE_NH;
        double z = b2[0];
        for (int j = 0; j < LINE_NH; ++j) {
            double a = b1[j];
            for (int k = 0; k < LINE_NF; ++k) a += W[j * LINE_NF + k] * f[k];
            z += w2[j] * (a > 0.0 ? a : 0.0);
        }
        out[2 + l] = 1.0 / (1.0 + exp(-z));
    }
}

/* Vertices of every event: pairs i < j (seed slots within the event) of kept
 * tracks (nhits > 0, score < score_max) with opposite seed charge, PCA by
 * orc_pca with g->newton_iters steps, kept if DOCA < doca_max.  Output is
 * event-major, (i, j)-ordered, at most `cap` per event; the number dropped
 * beyond the cap is returned in *overflow. */
int orc_vertex(const orc_geom *g, int n_events, const int *seed_off, const double *sqop, const double *x,
               const double *y, const double *tx, const double *ty, const double *qop, const double *score,
               const int *nhits, double score_max, int cap, int *count, int *vi, int *vj, double *vx, double *vy,
               double *vz, double *vdoca, double *vopen, long long *overflow, const double *line_w,
               double *extras /* nullable [E*cap*6] */)
{
    long long ovf = 0;
    for (int e = 0; e < n_events; ++e) {
        int s0 = seed_off[e], s1 = seed_off[e + 1];
        int m = 0;
        for (int i = s0; i < s1; ++i) {
            if (nhits[i] <= 0 || !(score[i] < score_max)) continue;
            for (int j = i + 1; j < s1; ++j) {
                if (nhits[j] <= 0 || !(score[j] < score_max)) continue;
                if ((sqop[i] > 0.0) == (sqop[j] > 0.0)) continue;
                double t1[5] = {x[i], y[i], tx[i], ty[i], qop[i]};
                double t2[5] = {x[j], y[j], tx[j], ty[j], qop[j]};
                double o[6];
                if (!orc_pca(g, t1, t2, g->newton_iters, o)) continue;
                if (!(o[3] < g->doca_max)) continue;
                if (m < cap) {
                    size_t k = (size_t)e * (size_t)cap + (size_t)m;
                    vi[k] = i - s0;
                    vj[k] = j - s0;
                    vx[k] = o[0];
                    vy[k] = o[1];
                    vz[k] = o[2];
                    vdoca[k] = o[3];
                    double d1[3] = {tx[i], ty[i], 1.0}, d2[3] = {tx[j], ty[j], 1.0}, c[3];
                    cross3(d1, d2, c);
                    vopen[k] = sqrt(dot3(c, c));
                    if (extras && line_w)
                        orc_vertex_extras(g, t1, t2, sqop[i], sqop[j], o[4], o[5], o, line_w, extras + 6 * k);
                } else {
                    ++ovf;
                }
                ++m;
            }
        }
        count[e] = m < cap ? m : cap;
    }
    *overflow = ovf;
    return 0;
}
