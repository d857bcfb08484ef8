// Device code of the Downstream tracking + two-track vertexing library for
// gfx950 (MI355X).  Included once, by ds_api.hip.
//
// Method (Kholoimov et al., arXiv:2503.13092):
//   * magnet-point (single kink) extrapolation of SciFi seeds to the UT
//     ("Algorithm Design", eq. 1 and the magnet-point text after it);
//   * Dv0 search: a first window in UTbX, then for each of up to 10 closest
//     UTbX hits a refined line through the hit and the magnet point, with the
//     closest UTaX hit and the two closest UTaU and UTbV hits;
//   * candidates scored by a least-squares chi2, best one per seed;
//   * ghost-killer MLP ("Ghost-Killer Neural Network");
//   * two-track vertexing: eq. 3/eq. 4 trajectories, Newton-Raphson PCA
//     ("Vertexing Two Downstream Tracks").
//
// Numerics.  Window searches, fits and vertex refinement run in float64 (on
// CDNA4 the float64 FMA rate equals the unpacked float32 rate), in the frame
// of the seed's un-kicked straight line x_S(z): a hit's residual is
// rho = u - c_L with c_L = x_S(z_L) - y(z_L)*tan(alpha_L).  In that frame the
// kinked prediction is MP*K*q/p*(z_M - z) and the refined line through a
// UTbX hit and the magnet point is rho_3*(z_M - z)/(z_M - z_3), because x_S
// passes through the magnet point.  The ghost-killer runs in float32 on
// features computed in float64 from the stored float32 track.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ds {

constexpr int NF = 17, NH1 = 32, NH2 = 16;
constexpr int NWEIGHTS = NH1 * NF + NH1 + NH2 * NH1 + NH2 + NH2 + 1;  // 1121
constexpr int MAX_L3 = 16;
constexpr int MAX_CLOSEST = 2;
constexpr int F_BAD_OFFSETS = 1, F_CAPACITY = 2, F_NONFINITE = 4;

// Geometry after host-side preprocessing (passed by value as a kernel argument).
struct DevGeom {
    double zl[4], tana[4];
    double zm, zs, zref;
    double mk;            // polarity * kick
    double inv_sigma2;
    double inv_5sigma;    // residual feature scale 1/(5 sigma)
    double w1c0, w1c1, w2c0, w2c1;
    double ffac[3];       // (z_M - z_L)/(z_M - z_3)
    double dz[4];         // z_L - z_ref
    // least-squares constants of the four valid layer sets {0,1,3}, {0,2,3}, {1,2,3}, {0,1,2,3}
    double fit_sz[4], fit_inv_det[4], fit_inv_n[4];
    double zm_ref, zm_seed, zref_seed;   // z_M - z_ref, z_M - z_seed, z_ref - z_seed
    double gc0, gc1, fp;                 // eq. 3
    double doca_max;
    float prescreen_thr2;                // (doca_max + margin)^2 for the float32 pair prescreen
    int max_l3;
    int ncl[3];
    int nw[3];                           // max(ncl, 1): radix of the candidate index
    int newton_iters;
};

struct TrackArgs {
    int n_events, n_seeds, n_hits, max_seeds, max_hits;
    const int *seed_off;
    const float *sx, *sy, *stx, *sty, *sqop;
    const int *hit_off;
    const float *hu;
    float *x, *y, *tx, *ty, *qop, *chi2, *score;
    int *h0, *h1, *h2, *h3, *nhits, *cand, *flags;
    int *counter;        // [0] next event, [1] finished workgroups (persistent launch)
    const float *W;      // ghost-killer parameters (resident)
    int fuse_mlp;
    int ev_single;       // >= 0: this launch processes only that event
    int hcap;            // LDS hit capacity of the launch
    int nb;              // bins per layer
    float u0, inv_bw;    // bin = floor((u - u0) * inv_bw), clamped
};

struct GhostArgs {
    int n_events, n_seeds, n_hits;
    const int *seed_off;
    const float *sx, *sy, *stx, *sty, *sqop;
    const int *hit_off;
    const float *hu;
    const float *x, *y, *tx, *ty, *qop, *chi2;
    const int *h0, *h1, *h2, *h3, *nhits;
    float *score;
    int *flags;
    const float *W;
};

struct VertexArgs {
    int n_events, n_seeds, max_seeds;
    const int *seed_off;
    const float *sqop;
    const float *x, *y, *tx, *ty, *qop, *score;
    const int *nhits;
    float score_max;
    int cap;
    int *count, *vi, *vj;
    float *vx, *vy, *vz, *vdoca;
    int *overflow, *flags;
    int *counter;        // [0] next event, [1] finished workgroups
    int ev_single;
    int tcap;            // LDS capacity for kept tracks
};

// ----------------------------------------------------------------- helpers

template <int BLOCK>
__device__ inline int block_exclusive_scan(int v, int *s_wsum, int *total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        int y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    if (lane == 63) s_wsum[wid] = x;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < BLOCK / 64; ++w) {
        int s = s_wsum[w];
        off += (w < wid) ? s : 0;
        tot += s;
    }
    __syncthreads();
    *total = tot;
    return off + x - v;
}

__device__ inline int bin_of(float u, float u0, float inv_bw, int nb)
{
    float t = (u - u0) * inv_bw;
    t = fminf(fmaxf(t, 0.0f), (float)(nb - 1));
    return (int)t;
}

__device__ inline bool finite5(float a, float b, float c, float d, float e)
{
    return isfinite(a) && isfinite(b) && isfinite(c) && isfinite(d) && isfinite(e);
}

// Walks outward from the insertion point of `m` in a sorted (u, index) run,
// returning positions in increasing (|u - m|, u, index) order while |u - m| <= W.
struct Walker {
    int lo, hi, left, right, run_cur, run_end;
};

__device__ inline void walker_init(Walker &w, const float *hu, const int *E, int layer, int nb, float u0,
                                   float inv_bw, double m)
{
    w.lo = E[layer * nb];
    w.hi = E[(layer + 1) * nb];
    int b = bin_of((float)m, u0, inv_bw, nb);
    int p = E[layer * nb + b];
    while (p > w.lo && (double)hu[p - 1] >= m) --p;
    while (p < w.hi && (double)hu[p] < m) ++p;
    w.left = p - 1;
    w.right = p;
    w.run_cur = 1;
    w.run_end = 0;
}

__device__ inline int walker_next(Walker &w, const float *hu, double m, double W)
{
    if (w.run_cur <= w.run_end) return w.run_cur++;
    double dl = (w.left >= w.lo) ? m - (double)hu[w.left] : INFINITY;
    double dr = (w.right < w.hi) ? (double)hu[w.right] - m : INFINITY;
    if (dl <= dr) {
        if (!(dl <= W)) return -1;
        // equal u on the left side: emit the run in index order
        float ul = hu[w.left];
        int q = w.left;
        while (q - 1 >= w.lo && hu[q - 1] == ul) --q;
        w.run_cur = q + 1;
        w.run_end = w.left;
        w.left = q - 1;
        return q;
    }
    if (!(dr <= W)) return -1;
    return w.right++;
}

// Least squares of residuals rho_L over a valid layer set (mask 11, 13, 14 or 15).
__device__ inline void fit_residuals(const DevGeom &G, int mask, const double rho[4], double &alpha, double &beta,
                                     double &chi2)
{
    int k = (mask == 15) ? 3 : (mask == 14) ? 2 : (mask == 13) ? 1 : 0;
    double sz = G.fit_sz[0], idet = G.fit_inv_det[0], in = G.fit_inv_n[0];
    sz = (k == 1) ? G.fit_sz[1] : sz;
    idet = (k == 1) ? G.fit_inv_det[1] : idet;
    in = (k == 1) ? G.fit_inv_n[1] : in;
    sz = (k == 2) ? G.fit_sz[2] : sz;
    idet = (k == 2) ? G.fit_inv_det[2] : idet;
    in = (k == 2) ? G.fit_inv_n[2] : in;
    sz = (k == 3) ? G.fit_sz[3] : sz;
    idet = (k == 3) ? G.fit_inv_det[3] : idet;
    in = (k == 3) ? G.fit_inv_n[3] : in;
    double sr = 0.0, szr = 0.0, n = 0.0;
#pragma unroll
    for (int L = 0; L < 4; ++L) {
        if ((mask >> L) & 1) {
            sr += rho[L];
            szr = fma(G.dz[L], rho[L], szr);
            n += 1.0;
        }
    }
    beta = (n * szr - sz * sr) * idet;
    alpha = (sr - beta * sz) * in;
    double c2 = 0.0;
#pragma unroll
    for (int L = 0; L < 4; ++L) {
        if ((mask >> L) & 1) {
            double r = rho[L] - alpha - beta * G.dz[L];
            c2 = fma(r, r, c2);
        }
    }
    chi2 = c2 * G.inv_sigma2;
}

// ------------------------------------------------------------ ghost-killer

// Features of a stored track (float32 values), its seed and its hits.
__device__ inline void ghost_features(const DevGeom &G, float xf, float yf, float txf, float tyf, float qf,
                                      float c2f, int nh, float sxf, float syf, float stxf, float styf, float sqf,
                                      const float hu4[4], int hasmask, float f[NF])
{
    f[0] = xf * 1e-3f;
    f[1] = yf * 1e-3f;
    f[2] = txf * (1.0f / 0.3f);
    f[3] = tyf * (1.0f / 0.3f);
    f[4] = qf * 2.0f;
    f[5] = c2f * 0.1f;
    f[6] = ((float)nh - 3.5f) * 2.0f;
    f[7] = sxf * (1.0f / 3000.0f);
    f[8] = syf * (1.0f / 3000.0f);
    f[9] = stxf * 2.0f;
    f[10] = styf * 2.0f;
    f[11] = sqf * 2.0f;
    const double x = xf, y = yf, tx = txf, ty = tyf;
#pragma unroll
    for (int L = 0; L < 4; ++L) {
        double r = 0.0;
        if ((hasmask >> L) & 1) {
            double yl = fma(ty, G.dz[L], y);
            double xhat = fma(yl, G.tana[L], (double)hu4[L]);
            r = (xhat - fma(tx, G.dz[L], x)) * G.inv_5sigma;
        }
        f[12 + L] = (float)r;
    }
    double xm_trk = fma(tx, G.zm_ref, x);
    double xm_seed = fma((double)stxf, G.zm_seed, (double)sxf);
    f[16] = (float)(xm_trk - xm_seed);
}

// Read-only, wave-uniform parameters: loads through the constant address
// space become scalar loads and the weights feed the FMAs as SGPR operands.
typedef const __attribute__((address_space(4))) float cfloat;

// 17 -> 32 ReLU -> 16 ReLU -> 1 sigmoid, float32 FMA; W is wave-uniform.
__device__ inline float mlp_score(const float *Wg, const float f[NF])
{
    // opaque to the optimiser: keeps the scalar weight loads next to their
    // uses instead of hoisting 1121 values out of the event loop into spills
    asm volatile("" : "+s"(Wg));
    cfloat *W = (cfloat *)(Wg);
    cfloat *W1 = W, *b1 = W + NH1 * NF, *W2 = b1 + NH1, *b2 = W2 + NH2 * NH1, *W3 = b2 + NH2, *b3 = W3 + NH2;
    float h1[NH1];
#pragma unroll
    for (int j = 0; j < NH1; ++j) {
        float a = b1[j];
#pragma unroll
        for (int k = 0; k < NF; ++k) a = fmaf(W1[j * NF + k], f[k], a);
        h1[j] = fmaxf(a, 0.0f);
    }
    float h2[NH2];
#pragma unroll
    for (int j = 0; j < NH2; ++j) {
        float a = b2[j];
#pragma unroll
        for (int k = 0; k < NH1; ++k) a = fmaf(W2[j * NH1 + k], h1[k], a);
        h2[j] = fmaxf(a, 0.0f);
    }
    float z = b3[0];
#pragma unroll
    for (int k = 0; k < NH2; ++k) z = fmaf(W3[k], h2[k], z);
    return 1.0f / (1.0f + __expf(-z));
}

// ------------------------------------------------------------------ track

__device__ inline void write_empty_track(const TrackArgs &a, int i)
{
    a.x[i] = 0.0f;
    a.y[i] = 0.0f;
    a.tx[i] = 0.0f;
    a.ty[i] = 0.0f;
    a.qop[i] = 0.0f;
    a.chi2[i] = 0.0f;
    if (a.fuse_mlp) a.score[i] = 0.0f;
    a.h0[i] = -1;
    a.h1[i] = -1;
    a.h2[i] = -1;
    a.h3[i] = -1;
    a.nhits[i] = 0;
    if (a.cand) a.cand[i] = -1;
}

// One seed, one lane: first window, refined windows, candidates, best.
__device__ inline void process_seed(const TrackArgs &a, const DevGeom &G, int i, const float *hu_s,
                                    const uint16_t *hidx_s, const int *E)
{
    const float fsx = a.sx[i], fsy = a.sy[i], fstx = a.stx[i], fsty = a.sty[i], fsq = a.sqop[i];
    if (!finite5(fsx, fsy, fstx, fsty, fsq)) {
        atomicOr(a.flags, F_NONFINITE);
        write_empty_track(a, i);
        return;
    }
    const double sx = fsx, sy = fsy, stx = fstx, sty = fsty, sq = fsq;
    double c[4];
#pragma unroll
    for (int L = 0; L < 4; ++L) {
        double dzs = G.zl[L] - G.zs;
        double xs = fma(stx, dzs, sx);
        double yl = fma(sty, dzs, sy);
        c[L] = fma(-yl, G.tana[L], xs);
    }
    const double aq = fabs(sq);
    const double W1 = fma(G.w1c1, aq, G.w1c0);
    const double W2 = fma(G.w2c1, aq, G.w2c0);
    const double m3 = c[3] + G.mk * sq * (G.zm - G.zl[3]);

    Walker w3;
    walker_init(w3, hu_s, E, 3, a.nb, a.u0, a.inv_bw, m3);
    int best_n = 0, best_c = -1;
    double best_chi2 = 0.0, best_alpha = 0.0, best_beta = 0.0;
    int bp0 = -1, bp1 = -1, bp2 = -1, bp3 = -1;

    for (int r3 = 0; r3 < G.max_l3; ++r3) {
        const int p3 = walker_next(w3, hu_s, m3, W1);
        if (p3 < 0) break;
        const double rho3 = (double)hu_s[p3] - c[3];
        int A[3][MAX_CLOSEST];
        int nA[3];
#pragma unroll
        for (int L = 0; L < 3; ++L) {
            const double mL = fma(rho3, G.ffac[L], c[L]);
            Walker wl;
            walker_init(wl, hu_s, E, L, a.nb, a.u0, a.inv_bw, mL);
            nA[L] = 0;
            A[L][0] = -1;
            A[L][1] = -1;
#pragma unroll
            for (int q = 0; q < MAX_CLOSEST; ++q) {
                if (q < G.ncl[L] && nA[L] == q) {
                    int p = walker_next(wl, hu_s, mL, W2);
                    if (p >= 0) {
                        A[L][q] = p;
                        nA[L] = q + 1;
                    }
                }
            }
        }
        double rho[4];
        rho[3] = rho3;
#pragma unroll
        for (int i0 = 0; i0 < MAX_CLOSEST; ++i0) {
            if (i0 >= (nA[0] > 0 ? nA[0] : 1)) continue;
            const int p0 = A[0][i0];
#pragma unroll
            for (int i1 = 0; i1 < MAX_CLOSEST; ++i1) {
                if (i1 >= (nA[1] > 0 ? nA[1] : 1)) continue;
                const int p1 = A[1][i1];
#pragma unroll
                for (int i2 = 0; i2 < MAX_CLOSEST; ++i2) {
                    if (i2 >= (nA[2] > 0 ? nA[2] : 1)) continue;
                    const int p2 = A[2][i2];
                    const int mask = 8 | (p0 >= 0 ? 1 : 0) | (p1 >= 0 ? 2 : 0) | (p2 >= 0 ? 4 : 0);
                    const int n = __popc(mask);
                    if (n < 3 || (p0 < 0 && p1 < 0)) continue;
                    rho[0] = p0 >= 0 ? (double)hu_s[p0] - c[0] : 0.0;
                    rho[1] = p1 >= 0 ? (double)hu_s[p1] - c[1] : 0.0;
                    rho[2] = p2 >= 0 ? (double)hu_s[p2] - c[2] : 0.0;
                    double al, be, c2;
                    fit_residuals(G, mask, rho, al, be, c2);
                    if (n > best_n || (n == best_n && c2 < best_chi2)) {
                        best_n = n;
                        best_chi2 = c2;
                        best_c = ((r3 * G.nw[0] + i0) * G.nw[1] + i1) * G.nw[2] + i2;
                        best_alpha = al;
                        best_beta = be;
                        bp0 = p0;
                        bp1 = p1;
                        bp2 = p2;
                        bp3 = p3;
                    }
                }
            }
        }
    }

    if (best_n == 0) {
        write_empty_track(a, i);
        return;
    }
    const double xs_ref = fma(stx, G.zref - G.zs, sx);
    const double ys_ref = fma(sty, G.zref - G.zs, sy);
    const float xf = (float)(xs_ref + best_alpha);
    const float txf = (float)(stx + best_beta);
    const float yf = (float)ys_ref;
    const float tyf = fsty;
    const float qf = (G.mk != 0.0) ? (float)(-best_beta / G.mk) : fsq;
    const float c2f = (float)best_chi2;
    a.x[i] = xf;
    a.y[i] = yf;
    a.tx[i] = txf;
    a.ty[i] = tyf;
    a.qop[i] = qf;
    a.chi2[i] = c2f;
    a.h0[i] = bp0 >= 0 ? (int)hidx_s[bp0] : -1;
    a.h1[i] = bp1 >= 0 ? (int)hidx_s[bp1] : -1;
    a.h2[i] = bp2 >= 0 ? (int)hidx_s[bp2] : -1;
    a.h3[i] = (int)hidx_s[bp3];
    a.nhits[i] = best_n;
    if (a.cand) a.cand[i] = best_c;
    if (a.fuse_mlp) {
        float hu4[4];
        hu4[0] = bp0 >= 0 ? hu_s[bp0] : 0.0f;
        hu4[1] = bp1 >= 0 ? hu_s[bp1] : 0.0f;
        hu4[2] = bp2 >= 0 ? hu_s[bp2] : 0.0f;
        hu4[3] = hu_s[bp3];
        const int has = (bp0 >= 0 ? 1 : 0) | (bp1 >= 0 ? 2 : 0) | (bp2 >= 0 ? 4 : 0) | 8;
        float f[NF];
        ghost_features(G, xf, yf, txf, tyf, qf, c2f, best_n, fsx, fsy, fstx, fsty, fsq, hu4, has, f);
        a.score[i] = mlp_score(a.W, f);
    }
}

// Stage one event's hits into LDS, bucket-sorted by (layer, bin) and sorted by
// (u, index) inside each bucket.  E[b] = start of bucket b, E[4*nb] = count.
// Hits are read once, HPT per lane per round with all loads in flight; the
// bucket slot returned by the counting atomic is kept to place the hit after
// the scan, so nothing is read twice.
template <int BLOCK>
__device__ inline bool stage_hits(const TrackArgs &a, int hb, const int hl[4], int nh, float *hu_s,
                                  uint16_t *hidx_s, int *E, int *s_bad, int *s_wsum)
{
    constexpr int HPT = 16;
    const int tid = threadIdx.x;
    const int NBT = 4 * a.nb;
    for (int k = tid; k <= NBT; k += BLOCK) E[k] = 0;
    if (tid == 0) *s_bad = 0;
    __syncthreads();
    const int rounds = (nh + HPT * BLOCK - 1) / (HPT * BLOCK);
    // events above HPT*BLOCK hits take several rounds; bucket counts accumulate across them
    for (int r = 0; r < rounds; ++r) {
        const int k0 = r * HPT * BLOCK + tid;
        float u[HPT];
#pragma unroll
        for (int j = 0; j < HPT; ++j) {
            const int k = k0 + j * BLOCK;
            u[j] = (k < nh) ? a.hu[hb + k] : 0.0f;
        }
        bool bad = false;
#pragma unroll
        for (int j = 0; j < HPT; ++j) {
            const int k = k0 + j * BLOCK;
            if (k < nh) {
                if (!isfinite(u[j])) {
                    bad = true;
                } else {
                    const int L = (k >= hl[1]) + (k >= hl[2]) + (k >= hl[3]);
                    atomicAdd(&E[L * a.nb + bin_of(u[j], a.u0, a.inv_bw, a.nb) + 1], 1);
                }
            }
        }
        if (bad) *s_bad = 1;
    }
    __syncthreads();
    if (*s_bad) return false;
    // exclusive scan of the bucket counts held at E[1..NBT]
    const int per = NBT / BLOCK;
    int local = 0;
    for (int j = 0; j < per; ++j) local += E[1 + tid * per + j];
    int tot;
    int run = block_exclusive_scan<BLOCK>(local, s_wsum, &tot);
    for (int j = 0; j < per; ++j) {
        int cnt = E[1 + tid * per + j];
        E[1 + tid * per + j] = run;
        run += cnt;
    }
    __syncthreads();
    for (int r = 0; r < rounds; ++r) {
        const int k0 = r * HPT * BLOCK + tid;
        float u[HPT];
#pragma unroll
        for (int j = 0; j < HPT; ++j) {
            const int k = k0 + j * BLOCK;
            u[j] = (k < nh) ? a.hu[hb + k] : 0.0f;
        }
#pragma unroll
        for (int j = 0; j < HPT; ++j) {
            const int k = k0 + j * BLOCK;
            if (k < nh) {
                const int L = (k >= hl[1]) + (k >= hl[2]) + (k >= hl[3]);
                const int pos = atomicAdd(&E[L * a.nb + bin_of(u[j], a.u0, a.inv_bw, a.nb) + 1], 1);
                hu_s[pos] = u[j];
                hidx_s[pos] = (uint16_t)(k - hl[L]);
            }
        }
    }
    __syncthreads();
    // (u, index) order inside each bucket
    for (int b = tid; b < NBT; b += BLOCK) {
        const int s = E[b], e = E[b + 1];
        for (int i = s + 1; i < e; ++i) {
            const float u = hu_s[i];
            const uint16_t id = hidx_s[i];
            int j = i - 1;
            while (j >= s && (hu_s[j] > u || (hu_s[j] == u && hidx_s[j] > id))) {
                hu_s[j + 1] = hu_s[j];
                hidx_s[j + 1] = hidx_s[j];
                --j;
            }
            hu_s[j + 1] = u;
            hidx_s[j + 1] = id;
        }
    }
    __syncthreads();
    return true;
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_track(TrackArgs a, DevGeom G)
{
    extern __shared__ __align__(16) unsigned char smem[];
    float *hu_s = reinterpret_cast<float *>(smem);
    uint16_t *hidx_s = reinterpret_cast<uint16_t *>(smem + (size_t)a.hcap * 4);
    int *E = reinterpret_cast<int *>(smem + (size_t)a.hcap * 6 + ((a.hcap * 6) & 15 ? 16 - ((a.hcap * 6) & 15) : 0));
    __shared__ int s_ev, s_bad;
    __shared__ int s_wsum[BLOCK / 64];
    const int tid = threadIdx.x;

    for (int iter = 0;; ++iter) {
        if (tid == 0) {
            int e;
            if (a.ev_single >= 0)
                e = (iter == 0) ? a.ev_single : a.n_events;
            else
                e = atomicAdd(&a.counter[0], 1);
            s_ev = e;
        }
        __syncthreads();
        const int e = s_ev;
        if (e >= a.n_events) break;

        const int s0 = a.seed_off[e], s1 = a.seed_off[e + 1];
        int ho[5];
#pragma unroll
        for (int L = 0; L < 5; ++L) ho[L] = a.hit_off[4 * e + L];
        bool seeds_ok = (0 <= s0) && (s0 <= s1) && (s1 <= a.n_seeds);
        bool hits_ok = (0 <= ho[0]) && (ho[4] <= a.n_hits);
#pragma unroll
        for (int L = 0; L < 4; ++L) hits_ok = hits_ok && (ho[L] <= ho[L + 1]) && (ho[L + 1] - ho[L] <= 65535);
        const int nh = ho[4] - ho[0];
        int bad = 0;
        if (!seeds_ok || !hits_ok) bad = F_BAD_OFFSETS;
        else if (nh > a.hcap || nh > a.max_hits || s1 - s0 > a.max_seeds) bad = F_CAPACITY;
        if (bad) {
            if (tid == 0) atomicOr(a.flags, bad);
            if (seeds_ok)
                for (int i = s0 + tid; i < s1; i += BLOCK) write_empty_track(a, i);
            __syncthreads();
            continue;
        }
        int hl[4];
#pragma unroll
        for (int L = 0; L < 4; ++L) hl[L] = ho[L] - ho[0];
        const bool staged = stage_hits<BLOCK>(a, ho[0], hl, nh, hu_s, hidx_s, E, &s_bad, s_wsum);
        if (!staged) {
            if (tid == 0) atomicOr(a.flags, F_NONFINITE);
            for (int i = s0 + tid; i < s1; i += BLOCK) write_empty_track(a, i);
            __syncthreads();
            continue;
        }
        for (int i = s0 + tid; i < s1; i += BLOCK) process_seed(a, G, i, hu_s, hidx_s, E);
        __syncthreads();
    }
    if (a.ev_single < 0 && tid == 0) {
        __threadfence();
        const int done = atomicAdd(&a.counter[1], 1);
        if (done == (int)gridDim.x - 1) {
            atomicExch(&a.counter[0], 0);
            atomicExch(&a.counter[1], 0);
            __threadfence();
        }
    }
}

// Standalone ghost-killer: one workgroup per event (grid-stride), lane per seed.
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_ghost(GhostArgs a, DevGeom G)
{
    for (int e = blockIdx.x; e < a.n_events; e += gridDim.x) {
        const int s0 = a.seed_off[e], s1 = a.seed_off[e + 1];
        int ho[5];
#pragma unroll
        for (int L = 0; L < 5; ++L) ho[L] = a.hit_off[4 * e + L];
        bool ok = (0 <= s0) && (s0 <= s1) && (s1 <= a.n_seeds) && (0 <= ho[0]) && (ho[4] <= a.n_hits);
#pragma unroll
        for (int L = 0; L < 4; ++L) ok = ok && (ho[L] <= ho[L + 1]);
        if (!ok) {
            if (threadIdx.x == 0) atomicOr(a.flags, F_BAD_OFFSETS);
            continue;
        }
        for (int i = s0 + (int)threadIdx.x; i < s1; i += BLOCK) {
            const int nh = a.nhits[i];
            if (nh <= 0) {
                a.score[i] = 0.0f;
                continue;
            }
            const int hh[4] = {a.h0[i], a.h1[i], a.h2[i], a.h3[i]};
            float hu4[4];
            int has = 0;
            bool hit_ok = true;
#pragma unroll
            for (int L = 0; L < 4; ++L) {
                hu4[L] = 0.0f;
                if (hh[L] >= 0) {
                    if (hh[L] < ho[L + 1] - ho[L]) {
                        hu4[L] = a.hu[ho[L] + hh[L]];
                        has |= 1 << L;
                    } else {
                        hit_ok = false;
                    }
                }
            }
            if (!hit_ok) {
                atomicOr(a.flags, F_BAD_OFFSETS);
                a.score[i] = 0.0f;
                continue;
            }
            float f[NF];
            ghost_features(G, a.x[i], a.y[i], a.tx[i], a.ty[i], a.qop[i], a.chi2[i], nh, a.sx[i], a.sy[i], a.stx[i],
                           a.sty[i], a.sqop[i], hu4, has, f);
            a.score[i] = mlp_score(a.W, f);
        }
    }
}

// ----------------------------------------------------------------- vertex

// Newton-Raphson point of closest approach in float64.  Offsets s, t are
// z - z_ref on each trajectory.  Returns false for (near-)parallel tracks or
// a singular Newton system.
__device__ inline bool pca64(const DevGeom &G, double x1, double y1, double tx1, double ty1, double g1, double x2,
                             double y2, double tx2, double ty2, double g2, double &vx, double &vy, double &vz,
                             double &doca)
{
    const double wx = x1 - x2, wy = y1 - y2;
    const double nx = ty1 - ty2, ny = tx2 - tx1, nz = tx1 * ty2 - ty1 * tx2;
    const double nn = nx * nx + ny * ny + nz * nz;
    if (nn < 1e-12) return false;
    // w x d = (wy, -wx, wx*ty - wy*tx) for w = (wx, wy, 0), d = (tx, ty, 1)
    const double inn = 1.0 / nn;
    const double base = wy * nx - wx * ny;
    double s = -(base + (wx * ty2 - wy * tx2) * nz) * inn;
    double t = -(base + (wx * ty1 - wy * tx1) * nz) * inn;
    for (int it = 0; it < G.newton_iters; ++it) {
        const double X1 = x1 + tx1 * s + g1 * s * s, Y1 = y1 + ty1 * s;
        const double X2 = x2 + tx2 * t + g2 * t * t, Y2 = y2 + ty2 * t;
        const double Dx = X1 - X2, Dy = Y1 - Y2, Dz = s - t;
        const double p1x = tx1 + 2.0 * g1 * s, p2x = tx2 + 2.0 * g2 * t;
        const double gr1 = Dx * p1x + Dy * ty1 + Dz;
        const double gr2 = -(Dx * p2x + Dy * ty2 + Dz);
        const double h11 = p1x * p1x + ty1 * ty1 + 1.0 + 2.0 * g1 * Dx;
        const double h22 = p2x * p2x + ty2 * ty2 + 1.0 - 2.0 * g2 * Dx;
        const double h12 = -(p1x * p2x + ty1 * ty2 + 1.0);
        const double det = h11 * h22 - h12 * h12;
        const double tr = h11 + h22;
        if (fabs(det) < 1e-12 * tr * tr) return false;
        const double idet = 1.0 / det;
        const double ds = (h22 * gr1 - h12 * gr2) * idet;
        const double dt = (h11 * gr2 - h12 * gr1) * idet;
        s -= ds;
        t -= dt;
    }
    const double X1 = x1 + tx1 * s + g1 * s * s, Y1 = y1 + ty1 * s;
    const double X2 = x2 + tx2 * t + g2 * t * t, Y2 = y2 + ty2 * t;
    const double Dx = X1 - X2, Dy = Y1 - Y2, Dz = s - t;
    vx = 0.5 * (X1 + X2);
    vy = 0.5 * (Y1 + Y2);
    vz = G.zref + 0.5 * (s + t);
    doca = sqrt(Dx * Dx + Dy * Dy + Dz * Dz);
    return true;
}

// Row-major rank k of the pair (a, b), a < b < n, back to (a, b).
__device__ inline void unrank_pair(int k, int n, int &pa, int &pb)
{
    const double tn = 2.0 * n - 1.0;
    int r = (int)floor((tn - sqrt(fmax(tn * tn - 8.0 * (double)k, 0.0))) * 0.5);
    r = max(0, min(r, n - 2));
    auto start = [n](int q) { return q * (2 * n - q - 1) / 2; };
    while (r + 1 <= n - 2 && start(r + 1) <= k) ++r;
    while (r > 0 && start(r) > k) --r;
    pa = r;
    pb = k - start(r) + r + 1;
}

template <int BLOCK, int PPT>
__global__ __launch_bounds__(BLOCK) void k_vertex(VertexArgs a, DevGeom G)
{
    constexpr int CH = BLOCK * PPT;
    extern __shared__ __align__(16) unsigned char smem[];
    float4 *st = reinterpret_cast<float4 *>(smem);                                  // x, y, tx, ty
    float *sq = reinterpret_cast<float *>(smem + (size_t)a.tcap * 16);              // track q/p
    int *sslot = reinterpret_cast<int *>(smem + (size_t)a.tcap * 20);               // slot << 1 | positive
    int *qk = reinterpret_cast<int *>(smem + (size_t)a.tcap * 24);                  // survivor pairs a << 16 | b
    float4 *qres = reinterpret_cast<float4 *>(smem + (size_t)a.tcap * 24 + CH * 4); // vx, vy, vz, doca
    int *qpass = reinterpret_cast<int *>(smem + (size_t)a.tcap * 24 + CH * 20);
    __shared__ int s_ev, s_n, s_out;
    __shared__ int s_wsum[BLOCK / 64];
    const int tid = threadIdx.x;
    const bool curved = (G.fp != 0.0);

    for (int iter = 0;; ++iter) {
        if (tid == 0) {
            int e;
            if (a.ev_single >= 0)
                e = (iter == 0) ? a.ev_single : a.n_events;
            else
                e = atomicAdd(&a.counter[0], 1);
            s_ev = e;
            s_n = 0;
            s_out = 0;
        }
        __syncthreads();
        const int e = s_ev;
        if (e >= a.n_events) break;
        const int s0 = a.seed_off[e], s1 = a.seed_off[e + 1];
        const bool ok = (0 <= s0) && (s0 <= s1) && (s1 <= a.n_seeds);
        if (!ok || s1 - s0 > a.tcap || s1 - s0 > a.max_seeds) {
            if (tid == 0) {
                atomicOr(a.flags, ok ? F_CAPACITY : F_BAD_OFFSETS);
                a.count[e] = 0;
            }
            __syncthreads();
            continue;
        }
        // kept tracks, compacted in slot order
        for (int base = s0; base < s1; base += BLOCK) {
            const int i = base + tid;
            int kept = 0;
            if (i < s1) kept = (a.nhits[i] > 0) && (a.score[i] < a.score_max);
            int tot;
            const int pos = block_exclusive_scan<BLOCK>(kept, s_wsum, &tot);
            if (kept) {
                const int k = s_n + pos;
                st[k] = make_float4(a.x[i], a.y[i], a.tx[i], a.ty[i]);
                sq[k] = a.qop[i];
                sslot[k] = ((i - s0) << 1) | (a.sqop[i] > 0.0f ? 1 : 0);
            }
            __syncthreads();
            if (tid == 0) s_n += tot;
            __syncthreads();
        }
        const int n = s_n;
        const int npairs = n * (n - 1) / 2;
        for (int chunk = 0; chunk < npairs; chunk += CH) {
            // stage 1: float32 prescreen of PPT consecutive pairs per lane
            const int k0 = chunk + tid * PPT;
            int pa = 0, pb = 0;
            if (k0 < npairs) unrank_pair(k0, n, pa, pb);
            int pairs[PPT];
            int bits = 0;
#pragma unroll
            for (int r = 0; r < PPT; ++r) {
                pairs[r] = (pa << 16) | pb;
                if (k0 + r < npairs) {
                    const int sa = sslot[pa], sb = sslot[pb];
                    bool surv = ((sa ^ sb) & 1) != 0;
                    if (surv && !curved) {
                        const float4 A = st[pa], B = st[pb];
                        const float wx = A.x - B.x, wy = A.y - B.y;
                        const float nx = A.w - B.w, ny = B.z - A.z;
                        const float nz = fmaf(A.z, B.w, -(A.w * B.z));
                        const float wn = fmaf(wx, nx, wy * ny);
                        const float nn = fmaf(nx, nx, fmaf(ny, ny, nz * nz));
                        surv = (nn < 1e-6f) || (wn * wn < G.prescreen_thr2 * nn);
                    }
                    bits |= (surv ? 1 : 0) << r;
                    ++pb;
                    if (pb == n) {
                        ++pa;
                        pb = pa + 1;
                    }
                }
            }
            int tot;
            int pos = block_exclusive_scan<BLOCK>(__popc(bits), s_wsum, &tot);
#pragma unroll
            for (int r = 0; r < PPT; ++r)
                if ((bits >> r) & 1) qk[pos++] = pairs[r];
            __syncthreads();
            // stage 2: float64 Newton refinement of the survivors
            for (int q = tid; q < tot; q += BLOCK) {
                const int ia = qk[q] >> 16, ib = qk[q] & 0xffff;
                const float4 A = st[ia], B = st[ib];
                const double g1 = -G.fp * (G.gc0 + G.gc1 * ((double)sq[ia] * 1e-3));
                const double g2 = -G.fp * (G.gc0 + G.gc1 * ((double)sq[ib] * 1e-3));
                double vx, vy, vz, dd;
                const bool good = pca64(G, A.x, A.y, A.z, A.w, g1, B.x, B.y, B.z, B.w, g2, vx, vy, vz, dd);
                const int pass = good && (dd < G.doca_max);
                qpass[q] = pass;
                qres[q] = make_float4((float)vx, (float)vy, (float)vz, (float)dd);
            }
            __syncthreads();
            // stage 3: ordered compaction of the passing pairs
            int cnt = 0;
#pragma unroll
            for (int r = 0; r < PPT; ++r) {
                const int q = tid * PPT + r;
                cnt += (q < tot) ? qpass[q] : 0;
            }
            int tot2;
            int opos = block_exclusive_scan<BLOCK>(cnt, s_wsum, &tot2);
            const int out0 = s_out;
#pragma unroll
            for (int r = 0; r < PPT; ++r) {
                const int q = tid * PPT + r;
                if (q < tot && qpass[q]) {
                    const int m = out0 + opos++;
                    if (m < a.cap) {
                        const size_t o = (size_t)e * (size_t)a.cap + (size_t)m;
                        const int ia = qk[q] >> 16, ib = qk[q] & 0xffff;
                        a.vi[o] = sslot[ia] >> 1;
                        a.vj[o] = sslot[ib] >> 1;
                        const float4 R = qres[q];
                        a.vx[o] = R.x;
                        a.vy[o] = R.y;
                        a.vz[o] = R.z;
                        a.vdoca[o] = R.w;
                    }
                }
            }
            __syncthreads();
            if (tid == 0) s_out += tot2;
            __syncthreads();
        }
        if (tid == 0) {
            const int m = s_out;
            a.count[e] = m < a.cap ? m : a.cap;
            if (m > a.cap) atomicAdd(a.overflow, m - a.cap);
        }
        __syncthreads();
    }
    if (a.ev_single < 0 && tid == 0) {
        __threadfence();
        const int done = atomicAdd(&a.counter[1], 1);
        if (done == (int)gridDim.x - 1) {
            atomicExch(&a.counter[0], 0);
            atomicExch(&a.counter[1], 0);
            __threadfence();
        }
    }
}

}  // namespace ds
