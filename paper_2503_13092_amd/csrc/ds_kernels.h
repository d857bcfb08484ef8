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
// Per-lane weight words of mlp_score_wave (lane l, group g = l / 16, n = l % 16):
// [u * 5 + s] = W1[16 u + n][4 s + g] (b1 in input column 17, zeros past it),
// [MLP_A2 + 4 u + r] = W2[n][16 u + 4 g + r], [MLP_B2 + r] = b2[4 g + r],
// [MLP_W3 + r] = W3[4 g + r], [MLP_B3] = b3; stored as float4 q of lane l at
// (q * 64 + l).
constexpr int MLP_K1 = 20, MLP_A2 = 10, MLP_B2 = 18, MLP_W3 = 22, MLP_B3 = 26;
constexpr int MLP_LANE_WORDS = 28;
constexpr int MLP_WM = 64 * MLP_LANE_WORDS;

// Host side: the per-lane order from the row-major parameters W1, b1, W2, b2, W3, b3.
inline void mlp_lane_layout(const float *w, float *wm)
{
    const float *W1 = w, *b1 = W1 + NH1 * NF, *W2 = b1 + NH1, *b2 = W2 + NH2 * NH1, *W3 = b2 + NH2, *b3 = W3 + NH2;
    for (int l = 0; l < 64; ++l) {
        const int g = l / 16, n = l % 16;
        float v[MLP_LANE_WORDS] = {};
        for (int u = 0; u < 2; ++u)
            for (int s = 0; s < MLP_K1 / 4; ++s) {
                const int j = 16 * u + n, k = 4 * s + g;
                v[u * (MLP_K1 / 4) + s] = k < NF ? W1[j * NF + k] : (k == NF ? b1[j] : 0.0f);
            }
        for (int u = 0; u < 2; ++u)
            for (int r = 0; r < 4; ++r) v[MLP_A2 + 4 * u + r] = W2[n * NH1 + 16 * u + 4 * g + r];
        for (int r = 0; r < 4; ++r) {
            v[MLP_B2 + r] = b2[4 * g + r];
            v[MLP_W3 + r] = W3[4 * g + r];
        }
        v[MLP_B3] = b3[0];
        for (int k = 0; k < MLP_LANE_WORDS; ++k) wm[((k / 4) * 64 + l) * 4 + k % 4] = v[k];
    }
}

constexpr int MAX_L3 = 16;
constexpr int MAX_CLOSEST = 2;
constexpr int F_BAD_OFFSETS = 1, F_CAPACITY = 2, F_NONFINITE = 4;
constexpr int LINE_NF = 12, LINE_NH = 32;
constexpr int LINE_NW = LINE_NH * LINE_NF + LINE_NH + LINE_NH + 1;  // 449 per network

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
    // Dv1 Y sectors: band k = [sec_y0 + k sec_h, sec_y0 + (k + 1) sec_h), k < nsec
    double sec_y0, sec_h, sec_tol;
    int nsec;
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
    int icap;            // LDS capacity for (seed, UTbX hit) items of one seed chunk
    // candidate-scoring mode: rows [n_seeds * cmax], row = seed * cmax + candidate index
    int cmax;
    int *r_seed, *r_cand, *r_nhits, *r_h0, *r_h1, *r_h2, *r_h3;
    float *r_x, *r_y, *r_tx, *r_ty, *r_qop, *r_chi2, *r_score;
    const float *Wrow;   // candidate rows: the ghost-killer weights W1, b1, W2, b2, W3, b3 row-major
    // fused vertexing (ds_process): kept tracks of an event go to LDS as they are written
    int tcap;            // LDS capacity for kept tracks of one event
    int krow_off;        // fused vertexing: byte offset in LDS of the row starts and descriptors (kept_rows_bytes)
    float score_max;
    int vcap;
    int *vcount, *vi, *vj;
    float *vx, *vy, *vz, *vdoca;
    int *voverflow, *vflags;
    float *m_pipi, *m_ppi, *line0, *line1, *line2, *line3;
    const float *WL;
    int nb;              // buckets of layers 0-2: u bins (Dv0) or sectors x u bins + 1 (Dv1)
    int nbu;             // u bins (per sector) of layers 0-2
    float u0, inv_bw;    // bin = floor((u - u0) * inv_bw), clamped to [0, nbu)
    int nb3, nbu3;       // the same for layer 3 (UTbX), stored after layers 0-2; Dv1 reads it
    float inv_bw3;       // by whole sectors only, so it has one u bin per sector
    const uint8_t *hsec; // Dv1: Y sector of every hit (null for Dv0)
    const int *order;    // persistent launch: events in this order (a permutation), null = input order
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

struct CloneArgs {
    int n_events, n_seeds, max_seeds;
    const int *seed_off;
    float *x, *y, *tx, *ty, *qop, *chi2, *score;
    int *h0, *h1, *h2, *h3, *nhits, *cand, *flags;
    int tcap;            // LDS capacity (seeds) per wavefront
};

struct VertexArgs {
    int n_events, n_seeds, max_seeds;
    const int *seed_off;
    const float *sqop;
    const float *x, *y, *tx, *ty, *qop, *score;
    const int *nhits;
    float score_max;
    int vcap;
    int *vcount, *vi, *vj;
    float *vx, *vy, *vz, *vdoca;
    int *voverflow, *flags;
    int *counter;        // [0] next event, [1] finished workgroups
    int ev_single;
    int tcap;            // LDS capacity for kept tracks
    // after-vertex outputs (nullable): masses (MeV) and the four trigger-line scores
    float *m_pipi, *m_ppi, *line0, *line1, *line2, *line3;
    const float *WL;     // trigger-line networks, 4 x (W1[32][12], b1[32], W2[32], b2)
};

// The tracking kernel's arguments as one block.
struct TrackKernArgs {
    TrackArgs a;
    DevGeom G;
};

// ----------------------------------------------------------------- helpers

// The launch's argument block, reached through an opaque copy of its address.
// Loads through the returned reference cannot move above the call, so a
// persistent kernel re-reads uniform arguments (scalar loads) in the phase that
// uses them instead of keeping all of them live, and spilled to vector lanes,
// across its whole loop.
template <typename T>
__device__ __forceinline__ const T &kernel_args()
{
    typedef const __attribute__((address_space(4))) T *cptr;
    cptr p = (cptr)__builtin_amdgcn_kernarg_segment_ptr();
    asm volatile("" : "+s"(p));
    return *(const T *)p;
}

// Workgroup barrier ordering LDS traffic only: unlike __syncthreads it does not
// wait for the wave's outstanding global stores.
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Inclusive sum over the 64 lanes of a wavefront, in lane order: four doubling
// row shifts within rows of 16 lanes, then the row broadcasts of lanes 15 and
// 31 (DPP, no LDS traffic).  Lanes outside a shift's source read 0.
__device__ __forceinline__ int wave_inclusive_sum(int x)
{
    x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, false);   // row_shr:1
    x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, false);   // row_shr:2
    x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, false);   // row_shr:4
    x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, false);   // row_shr:8
    x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false);   // row_bcast:15 into rows 1, 3
    x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false);   // row_bcast:31 into rows 2, 3
    return x;
}

template <int BLOCK>
__device__ __forceinline__ int block_exclusive_scan(int v, int *s_wsum, int *total)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int x = wave_inclusive_sum(v);
    if (lane == 63) s_wsum[wid] = x;
    lds_barrier();
    int off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < BLOCK / 64; ++w) {
        int s = s_wsum[w];
        off += (w < wid) ? s : 0;
        tot += s;
    }
    lds_barrier();
    *total = tot;
    return off + x - v;
}

__device__ __forceinline__ int bin_of(float u, float u0, float inv_bw, int nb)
{
    float t = (u - u0) * inv_bw;
    t = fminf(fmaxf(t, 0.0f), (float)(nb - 1));
    return (int)t;
}

__device__ __forceinline__ bool finite5(float a, float b, float c, float d, float e)
{
    return isfinite(a) && isfinite(b) && isfinite(c) && isfinite(d) && isfinite(e);
}

// Window order of hits: (|u - m|, u, index within the layer run), lexicographic.
__device__ __forceinline__ bool key_less(double da, float ua, int ia, double db, float ub, int ib)
{
    return da < db || (da == db && (ua < ub || (ua == ub && ia < ib)));
}

// Window order of the hit at LDS position p (distance d, coordinate u) against
// the kept hit at position pk (distance dk; pk < 0: empty slot).
__device__ __forceinline__ bool before(const float *hu_s, const uint16_t *hidx_s, double d, float u, int p, double dk, int pk)
{
    if (d != dk || pk < 0) return d < dk || pk < 0;
    const float uk = hu_s[pk];
    if (u != uk) return u < uk;
    return hidx_s[p] < hidx_s[pk];
}

// The window's bin bounds in float32: m and W rounded (errors below 1e-4 mm
// for |m| < 2000 mm) and widened by 1e-3 mm, so the buckets always cover
// [m - W, m + W] (a superset: membership is decided on |u - m| <= W in float64).
__device__ __forceinline__ void window_bins(double m, double W, float u0, float inv_bw, int nb, int &b_lo, int &b_hi)
{
    const float mf = (float)m, wf = (float)W + 1e-3f;
    b_lo = bin_of(mf - wf, u0, inv_bw, nb);
    b_hi = bin_of(mf + wf, u0, inv_bw, nb);
}

// LDS positions [p_lo, p_hi) of the buckets of `layer` covering [m - W, m + W]
// (a superset of the window: membership is decided on |u - m| <= W).
__device__ __forceinline__ void bin_range(const uint16_t *E, int layer, int nb, float u0, float inv_bw, double m, double W,
                                 int &p_lo, int &p_hi)
{
    int b_lo, b_hi;
    window_bins(m, W, u0, inv_bw, nb, b_lo, b_hi);
    p_lo = E[layer * nb + b_lo];
    p_hi = E[layer * nb + b_hi + 1];
}

// Candidate key for the per-seed reduction: more hits first, then lower chi2
// (non-negative double bits are monotone; the 8 lowest mantissa bits are
// dropped), then lower candidate index.
__device__ __forceinline__ unsigned long long pack_key(int n, double chi2, int c)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(chi2);
    return ((unsigned long long)(4 - n) << 63) | ((b >> 8) << 7) | (unsigned long long)c;
}

struct SeedConst {
    double c[4];     // c_L = x_S(z_L) - y(z_L) tan(alpha_L)
    float q;         // seed q/p (window widths and the kinked prediction)
    uint16_t lo, hi; // LDS range of the UTbX buckets covering the first window
};

// Least-squares constants of one valid layer set (mask 11, 13, 14 or 15):
// sum of dz, 1/det of the normal equations, 1/n, and the 0/1 layer weights.
struct FitConst {
    double sz, idet, in, n;
    double w[4];
};

__device__ __forceinline__ FitConst fit_const(const DevGeom &G, int mask)
{
    const int k = (mask == 15) ? 3 : (mask == 14) ? 2 : (mask == 13) ? 1 : 0;
    FitConst f;
    f.sz = G.fit_sz[0];
    f.idet = G.fit_inv_det[0];
    f.in = G.fit_inv_n[0];
#pragma unroll
    for (int j = 1; j < 4; ++j) {
        f.sz = (k == j) ? G.fit_sz[j] : f.sz;
        f.idet = (k == j) ? G.fit_inv_det[j] : f.idet;
        f.in = (k == j) ? G.fit_inv_n[j] : f.in;
    }
    f.n = (mask == 15) ? 4.0 : 3.0;
#pragma unroll
    for (int L = 0; L < 4; ++L) f.w[L] = ((mask >> L) & 1) ? 1.0 : 0.0;
    return f;
}

// Straight-line least squares rho_L ~ alpha + beta dz_L over the layer set of
// f; rho_L must be 0 for a layer outside the set (it then adds nothing to the
// sums, and its weight 0 keeps it out of chi2).
__device__ __forceinline__ void fit_set(const DevGeom &G, const FitConst &f, const double rho[4], double &alpha,
                               double &beta, double &chi2)
{
    double sr = 0.0, szr = 0.0;
#pragma unroll
    for (int L = 0; L < 4; ++L) {
        sr += rho[L];
        szr = fma(G.dz[L], rho[L], szr);
    }
    beta = (f.n * szr - f.sz * sr) * f.idet;
    alpha = (sr - beta * f.sz) * f.in;
    double c2 = 0.0;
#pragma unroll
    for (int L = 0; L < 4; ++L) {
        const double r = rho[L] - alpha - beta * G.dz[L];
        c2 = fma(r, r * f.w[L], c2);
    }
    chi2 = c2 * G.inv_sigma2;
}

// ------------------------------------------------------------ ghost-killer

// Features of a stored track (float32 values), its seed and its hits.
__device__ __forceinline__ void ghost_features(const DevGeom &G, float xf, float yf, float txf, float tyf, float qf,
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

// The ghost-killer network of one lane on the vector ALUs, its weights read
// through the scalar cache (the same for every lane): for rows produced one at
// a time in divergent code, where the wavefront network cannot run.  Hidden
// layer 1 is consumed as it is produced (h2 accumulates over it in unit order).
__device__ __forceinline__ float mlp_score_lane(const float *Wg, const float f[NF])
{
    asm volatile("" : "+s"(Wg));   // keeps the weight loads beside their uses
    cfloat *W1 = (cfloat *)(Wg), *b1 = W1 + NH1 * NF, *W2 = b1 + NH1, *b2 = W2 + NH2 * NH1, *W3 = b2 + NH2,
           *b3 = W3 + NH2;
    float h2[NH2];
#pragma unroll
    for (int k = 0; k < NH2; ++k) h2[k] = b2[k];
#pragma unroll
    for (int j = 0; j < NH1; ++j) {
        float z = b1[j];
#pragma unroll
        for (int k = 0; k < NF; ++k) z = fmaf(W1[j * NF + k], f[k], z);
        const float h = fmaxf(z, 0.0f);
#pragma unroll
        for (int k = 0; k < NH2; ++k) h2[k] = fmaf(W2[k * NH1 + j], h, h2[k]);
    }
    float z = b3[0];
#pragma unroll
    for (int k = 0; k < NH2; ++k) z = fmaf(W3[k], fmaxf(h2[k], 0.0f), z);
    return 1.0f / (1.0f + __expf(-z));
}

// 17 -> 32 ReLU -> 16 ReLU -> 1 sigmoid, float32 FMA; W is wave-uniform.
// The ghost-killer network ("Ghost-Killer Neural Network": 17 inputs, ReLU
// hidden layers of 32 and 16, sigmoid output) of a wavefront's 64 rows, one
// row per lane, on the matrix cores.  Both hidden layers are products
// H^T = W X^T of v_mfma_f32_16x16x4_f32 tiles: 16 units x 16 rows per tile,
// 4 inputs per step.  In a tile, lane l holds row (l % 16) of its block and
// input / unit index 4 (l / 16) + r, so a lane's own 17 features are first
// transposed across the four 16-lane groups (permlane swaps), and the layer-1
// output is already in the layer-2 operand layout.  The weights come in the
// per-lane order built by mlp_lane_layout.  Every output element is the same
// sequence of operations wherever its row sits, so a track's score does not
// depend on its lane.
typedef float f32x4 __attribute__((ext_vector_type(4)));

// lanes 32..63 of a <-> lanes 0..31 of b
__device__ __forceinline__ void lane_swap32(float &a, float &b)
{
    const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    a = __uint_as_float(r[0]);
    b = __uint_as_float(r[1]);
}

// odd 16-lane groups of a <-> even 16-lane groups of b
__device__ __forceinline__ void lane_swap16(float &a, float &b)
{
    const auto r = __builtin_amdgcn_permlane16_swap(__float_as_uint(a), __float_as_uint(b), false, false);
    a = __uint_as_float(r[0]);
    b = __uint_as_float(r[1]);
}

// This lane's weight words of mlp_score_wave.
__device__ __forceinline__ void mlp_lane_weights(const float *Wm, float w[MLP_LANE_WORDS])
{
    const int lane = threadIdx.x & 63;
    const float4 *W4 = reinterpret_cast<const float4 *>(Wm);
#pragma unroll
    for (int q = 0; q < MLP_LANE_WORDS / 4; ++q) {
        const float4 v = W4[q * 64 + lane];
        w[4 * q] = v.x;
        w[4 * q + 1] = v.y;
        w[4 * q + 2] = v.z;
        w[4 * q + 3] = v.w;
    }
}

// The network on operands already in the MFMA layout: x[4 s + b] holds, in
// 16-lane group j, input 4 s + j of the row of lane 16 b + l % 16 (inputs past
// the 17 features: the bias column 1, then zeros; all zeros for rows without
// a track); rows: the ballot of the lanes with a row.  All 64 lanes call it
// together.
__device__ __forceinline__ float mlp_core(const float w[MLP_LANE_WORDS], const float x[MLP_K1], unsigned long long rows)
{
    const int grp = (threadIdx.x & 63) >> 4;
    float z = 0.0f;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        if (((rows >> (16 * b)) & 0xffffull) == 0) continue;   // no row in this block
        f32x4 h[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            h[u] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int s = 0; s < MLP_K1 / 4; ++s)
                h[u] = __builtin_amdgcn_mfma_f32_16x16x4f32(w[u * (MLP_K1 / 4) + s], x[4 * s + b], h[u], 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 4; ++r) h[u][r] = fmaxf(h[u][r], 0.0f);
        }
        f32x4 o = f32x4{w[MLP_B2], w[MLP_B2 + 1], w[MLP_B2 + 2], w[MLP_B2 + 3]};
#pragma unroll
        for (int u = 0; u < 2; ++u)
#pragma unroll
            for (int r = 0; r < 4; ++r)
                o = __builtin_amdgcn_mfma_f32_16x16x4f32(w[MLP_A2 + 4 * u + r], h[u][r], o, 0, 0, 0);
        float p = 0.0f;
#pragma unroll
        for (int r = 0; r < 4; ++r) p = fmaf(w[MLP_W3 + r], fmaxf(o[r], 0.0f), p);
        // sum over the four groups: (g0 + g2) + (g1 + g3), in every group
        float c = p, d = p;
        lane_swap32(c, d);
        const float p2 = c + d;
        c = p2;
        d = p2;
        lane_swap16(c, d);
        const float zb = c + d;
        z = grp == b ? zb : z;
    }
    z += w[MLP_B3];
    return 1.0f / (1.0f + __expf(-z));
}

// The network on each lane's own 17 features f (registers).  All 64 lanes
// must call it together (wave-uniform control flow).  Lanes with row == false
// contribute zeros; every lane gets its own row's score.
__device__ __forceinline__ float mlp_score_wave(const float w[MLP_LANE_WORDS], const float f[NF], bool row)
{
    const unsigned long long rows = __ballot(row);
    // layer-1 inputs padded to 20: the features, 1 (the bias column), zeros
    float x[MLP_K1];
#pragma unroll
    for (int k = 0; k < MLP_K1; ++k) x[k] = (row && k < NF) ? f[k] : (row && k == NF) ? 1.0f : 0.0f;
    // per step s, (register 4s + j, group b) -> (register 4s + b, group j): then
    // x[4s + b] holds, in group j, input 4s + j of the row of lane 16 b + l % 16
#pragma unroll
    for (int s = 0; s < MLP_K1 / 4; ++s) {
        lane_swap32(x[4 * s], x[4 * s + 2]);
        lane_swap32(x[4 * s + 1], x[4 * s + 3]);
        lane_swap16(x[4 * s], x[4 * s + 1]);
        lane_swap16(x[4 * s + 2], x[4 * s + 3]);
    }
    return mlp_core(w, x, rows);
}

// A wavefront's feature tile in LDS, already in the operand layout: feature k
// of the row of lane l at T[k * 64 + 4 (l % 16) + l / 16], so that a lane of
// group j reads inputs 4 s + j of its four row blocks as one 16-byte word.
constexpr int MLP_TILE = NF * 64;   // floats per wavefront

__device__ __forceinline__ int mlp_tile_pos(int lane) { return 4 * (lane & 15) + (lane >> 4); }

// Row of this lane into the tile (zeros for a lane without a row).
__device__ __forceinline__ void mlp_tile_store(float *T, const float f[NF], bool row)
{
    const int pos = mlp_tile_pos(threadIdx.x & 63);
#pragma unroll
    for (int k = 0; k < NF; ++k) T[k * 64 + pos] = row ? f[k] : 0.0f;
}

// The network on the wavefront's tile T (written by mlp_tile_store of every
// lane of this wavefront: a wavefront's LDS operations complete in order).
__device__ __forceinline__ float mlp_score_tile(const float w[MLP_LANE_WORDS], const float *T, bool row)
{
    const int lane = threadIdx.x & 63, grp = lane >> 4, r = lane & 15;
    const unsigned long long rows = __ballot(row);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);   // the tile's stores stay ahead of the loads
    float x[MLP_K1];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const f32x4 v = *reinterpret_cast<const f32x4 *>(T + (4 * s + grp) * 64 + 4 * r);
#pragma unroll
        for (int b = 0; b < 4; ++b) x[4 * s + b] = v[b];
    }
    // inputs 16..19: feature 16 (group 0), the bias column (group 1), zeros
    const f32x4 v = *reinterpret_cast<const f32x4 *>(T + 16 * 64 + 4 * r);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const float bias = ((rows >> (16 * b + r)) & 1ull) ? 1.0f : 0.0f;
        x[16 + b] = grp == 0 ? v[b] : (grp == 1 ? bias : 0.0f);
    }
    return mlp_core(w, x, rows);
}

// ------------------------------------------------------------------ track

__device__ __forceinline__ void write_empty_track(const TrackArgs &a, int i)
{
    if (!a.x) return;  // candidate-scoring mode writes no track slots
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

// First-window centre in UTbX: the kinked prediction of the seed.  One
// expression for every use, so that membership tests agree bit for bit.
__device__ __forceinline__ double window1_centre(const DevGeom &G, double c3, double q)
{
    return fma(G.mk * q, G.zm - G.zl[3], c3);
}

// Seed constants of the residual frame and the first-window centre / width.
__device__ __forceinline__ bool seed_frame(const DevGeom &G, float fsx, float fsy, float fstx, float fsty, float fsq,
                                  SeedConst &sc, double &m3, double &W1)
{
    if (!finite5(fsx, fsy, fstx, fsty, fsq)) return false;
    const double sx = fsx, sy = fsy, stx = fstx, sty = fsty, sq = fsq;
#pragma unroll
    for (int L = 0; L < 4; ++L) {
        const double dzs = G.zl[L] - G.zs;
        const double xs = fma(stx, dzs, sx);
        const double yl = fma(sty, dzs, sy);
        sc.c[L] = fma(-yl, G.tana[L], xs);
    }
    sc.q = fsq;
    W1 = fma(G.w1c1, fabs(sq), G.w1c0);
    m3 = window1_centre(G, sc.c[3], sq);
    return true;
}

// ------------------------------------------------------------------ Dv1

// Y sectors compatible with height y: those whose band
// [y0 + k h, y0 + (k + 1) h) overlaps [y - tol, y + tol]; klo > khi (15, 0)
// when none does.  The same division and floor as the definition.
__device__ __forceinline__ void sector_range(const DevGeom &G, double y, int &klo, int &khi)
{
    const double a = (y - G.sec_tol - G.sec_y0) / G.sec_h;
    const double b = (y + G.sec_tol - G.sec_y0) / G.sec_h;
    const double fa = floor(a), fb = floor(b), top = (double)(G.nsec - 1);
    if (fb < 0.0 || fa > top) {
        klo = 15;
        khi = 0;
        return;
    }
    klo = fa < 0.0 ? 0 : (int)fa;
    khi = fb > top ? G.nsec - 1 : (int)fb;
}

// Dv1 keeps the four layers' sector ranges in the seed constants, 4 + 4 bits
// per layer (lo: layers 0 and 1, hi: layers 2 and 3).
__device__ __forceinline__ void seed_sectors(const DevGeom &G, float fsy, float fsty, SeedConst &sc)
{
    uint32_t packed = 0;
#pragma unroll
    for (int L = 0; L < 4; ++L) {
        const double yl = fma((double)fsty, G.zl[L] - G.zs, (double)fsy);
        int klo, khi;
        sector_range(G, yl, klo, khi);
        packed |= (uint32_t)(klo | (khi << 4)) << (8 * L);
    }
    sc.lo = (uint16_t)(packed & 0xffffu);
    sc.hi = (uint16_t)(packed >> 16);
}

__device__ __forceinline__ void sector_span(const SeedConst &sc, int L, int &klo, int &khi)
{
    const uint32_t v = (((uint32_t)sc.lo | ((uint32_t)sc.hi << 16)) >> (8 * L)) & 0xffu;
    klo = (int)(v & 15u);
    khi = (int)(v >> 4);
}

// LDS ranges of the buckets of layer L, sectors klo..khi (at most two), whose
// u bins cover [m - W, m + W]; buckets are (layer, sector, u bin).  Branch-free:
// the four bounds are read at sector indices clamped into the layer's buckets
// and dropped when the sector is not in the span.
__device__ __forceinline__ void sector_bins(const uint16_t *E, const TrackArgs &a, int nsec, int L, int klo, int khi, double m,
                                   double W, int &lo0, int &len0, int &lo1, int &len1)
{
    int b_lo, b_hi;
    window_bins(m, W, a.u0, a.inv_bw, a.nbu, b_lo, b_hi);
    const int base0 = L * a.nb + min(klo, nsec - 1) * a.nbu, base1 = L * a.nb + min(klo + 1, nsec - 1) * a.nbu;
    const int e0 = E[base0 + b_lo], e1 = E[base0 + b_hi + 1], e2 = E[base1 + b_lo], e3 = E[base1 + b_hi + 1];
    const bool in0 = klo <= khi, in1 = klo + 1 <= khi;
    lo0 = in0 ? e0 : 0;
    len0 = in0 ? e1 - e0 : 0;
    lo1 = in1 ? e2 : 0;
    len1 = in1 ? e3 - e2 : 0;
}

// Does the line through the magnet point and the UTbX hit at p3 meet a UTaX
// hit of a compatible sector within W (the axial triplet)?  In two parts: the
// probe of the first two UTaX positions (most probes look at <= 2 hits),
// straight-line so that two seeds' probes can overlap, then the rest.
constexpr int DV1_PROBE = 4;   // window positions read by the paired probe

struct TripletProbe {
    double m0;
    int lo0, len0, lo1, len1;
    bool hit;
};

__device__ __forceinline__ TripletProbe dv1_probe(const DevGeom &G, const TrackArgs &a, const float *hu_s, const uint16_t *E,
                                         const SeedConst &sc, int k0lo, int k0hi, double W, int p3)
{
    TripletProbe t;
    t.m0 = fma((double)hu_s[p3] - sc.c[3], G.ffac[0], sc.c[0]);
    sector_bins(E, a, G.nsec, 0, k0lo, k0hi, t.m0, W, t.lo0, t.len0, t.lo1, t.len1);
    const int n = t.len0 + t.len1;
    const int pa = t.len0 > 0 ? t.lo0 : t.lo1, pb = t.len0 > 1 ? t.lo0 + 1 : (t.len0 == 1 ? t.lo1 : t.lo1 + 1);
    const float ua = hu_s[n > 0 ? pa : 0], ub = hu_s[n > 1 ? pb : 0];
    // bitwise, not short-circuit: no branch between the reads and the tests
    t.hit = ((n > 0) & (fabs((double)ua - t.m0) <= W)) | ((n > 1) & (fabs((double)ub - t.m0) <= W));
    return t;
}

// Probes of two (seed, UTbX hit) pairs, stage by stage (the hits' u, the
// projections, the eight bucket bounds, the first four UTaX positions of each
// window), so that each stage costs one LDS round trip for both; a window
// holding more than four hits is finished by dv1_rest.
__device__ __forceinline__ void dv1_probe_pair(const DevGeom &G, const TrackArgs &a, const float *hu_s, const uint16_t *E,
                                      const SeedConst &sa, const SeedConst &sb, int ka_lo, int ka_hi, int kb_lo,
                                      int kb_hi, double Wa, double Wb, int pa3, int pb3, TripletProbe &ta,
                                      TripletProbe &tb)
{
    const float ua3 = hu_s[pa3], ub3 = hu_s[pb3];
    ta.m0 = fma((double)ua3 - sa.c[3], G.ffac[0], sa.c[0]);
    tb.m0 = fma((double)ub3 - sb.c[3], G.ffac[0], sb.c[0]);
    sector_bins(E, a, G.nsec, 0, ka_lo, ka_hi, ta.m0, Wa, ta.lo0, ta.len0, ta.lo1, ta.len1);
    sector_bins(E, a, G.nsec, 0, kb_lo, kb_hi, tb.m0, Wb, tb.lo0, tb.len0, tb.lo1, tb.len1);
    const int na = ta.len0 + ta.len1, nb = tb.len0 + tb.len1;
    float va[DV1_PROBE], vb[DV1_PROBE];
#pragma unroll
    for (int k = 0; k < DV1_PROBE; ++k) {
        const int qa = k < ta.len0 ? ta.lo0 + k : ta.lo1 + (k - ta.len0);
        const int qb = k < tb.len0 ? tb.lo0 + k : tb.lo1 + (k - tb.len0);
        va[k] = hu_s[k < na ? qa : 0];
        vb[k] = hu_s[k < nb ? qb : 0];
    }
    bool ha = false, hb = false;
#pragma unroll
    for (int k = 0; k < DV1_PROBE; ++k) {
        ha |= (k < na) & (fabs((double)va[k] - ta.m0) <= Wa);
        hb |= (k < nb) & (fabs((double)vb[k] - tb.m0) <= Wb);
    }
    ta.hit = ha;
    tb.hit = hb;
}

__device__ __forceinline__ bool dv1_rest(const float *hu_s, const TripletProbe &t, double W, int from)
{
    bool hit = t.hit;
    const int n = t.len0 + t.len1;
    for (int k = from; k < n && !hit; ++k) {
        const int p = k < t.len0 ? t.lo0 + k : t.lo1 + (k - t.len0);
        hit = fabs((double)hu_s[p] - t.m0) <= W;
    }
    return hit;
}

__device__ __forceinline__ bool dv1_triplet(const DevGeom &G, const TrackArgs &a, const float *hu_s, const uint16_t *E,
                                   const SeedConst &sc, int k0lo, int k0hi, double W, int p3)
{
    return dv1_rest(hu_s, dv1_probe(G, a, hu_s, E, sc, k0lo, k0hi, W, p3), W, 2);
}

// Candidate key of Dv1: the candidate index holds the UTbX hit's index in its
// layer run, 20 bits; 43 bits of chi2 above it.
__device__ __forceinline__ unsigned long long pack_key_dv1(int n, double chi2, int c)
{
    const unsigned long long b = (unsigned long long)__double_as_longlong(chi2);
    return ((unsigned long long)(4 - n) << 63) | ((b >> 20) << 20) | (unsigned long long)c;
}

// Every valid candidate through one UTbX hit (rank r3, LDS position p3), in
// candidate-index order: refined windows in UTaX, UTaU, UTbV, the <= 4 option
// tuples, their fits.  visit(n, c, alpha, beta, chi2, bp) is called for each.
template <int N0, int N1, int N2, bool DV1, typename Visit>
__device__ __forceinline__ void item_candidates_n(const DevGeom &G, const TrackArgs &a, const float *hu_s,
                                       const uint16_t *hidx_s, const uint16_t *E, const SeedConst &sc, int cb, int p3,
                                       Visit &&visit)
{
    const double W2 = fma(G.w2c1, fabs((double)sc.q), G.w2c0);
    const double rho3 = (double)hu_s[p3] - sc.c[3];
    double m[3];
    // per layer, up to two LDS ranges (Dv1: one per compatible Y sector)
    int lo[3], len[3], lo1[3] = {0, 0, 0}, len0[3];
    int maxlen = 0;
#pragma unroll
    for (int L = 0; L < 3; ++L) {
        m[L] = fma(rho3, G.ffac[L], sc.c[L]);
        if (DV1) {
            int klo, khi, l1;
            sector_span(sc, L, klo, khi);
            sector_bins(E, a, G.nsec, L, klo, khi, m[L], W2, lo[L], len0[L], lo1[L], l1);
            len[L] = len0[L] + l1;
        } else {
            int hi;
            bin_range(E, L, a.nb, a.u0, a.inv_bw, m[L], W2, lo[L], hi);
            len[L] = hi - lo[L];
            len0[L] = len[L];
        }
        maxlen = max(maxlen, len[L]);
    }
    // the three layers advance together: one LDS round trip per step.  The
    // kept hits are held as (float32-rounded |delta|, LDS position): rounding
    // is monotone, so a strictly smaller rounded distance is a strictly
    // smaller distance; equal rounded distances (exact ties included) are
    // settled on the full key (|delta| in float64, u, index, re-read from LDS)
    // on a path of their own, taken by the whole wavefront when any lane
    // needs it.  Window membership is always the float64 test.
    float f0[3] = {INFINITY, INFINITY, INFINITY}, f1[3] = {INFINITY, INFINITY, INFINITY};
    int p0k[3] = {-1, -1, -1}, p1k[3] = {-1, -1, -1};
    for (int k = 0; k < maxlen; ++k) {
        // the three loads first (a finished layer re-reads its start), then the tests
        int pp[3];
        float uu[3];
#pragma unroll
        for (int L = 0; L < 3; ++L) {
            const int kk = k < len[L] ? k : 0;
            pp[L] = (!DV1 || kk < len0[L]) ? lo[L] + kk : lo1[L] + (kk - len0[L]);
            uu[L] = hu_s[pp[L]];
        }
        double dd[3];
        float fd[3];
        bool in[3], lt0[3], lt1[3], eq[3];
        bool any_eq = false;
#pragma unroll
        for (int L = 0; L < 3; ++L) {
            const int NL = L == 0 ? N0 : (L == 1 ? N1 : N2);
            dd[L] = fabs((double)uu[L] - m[L]);
            fd[L] = (float)dd[L];
            in[L] = (k < len[L]) & (dd[L] <= W2);
            lt0[L] = in[L] & (fd[L] < f0[L]);
            lt1[L] = (NL > 1) & in[L] & !lt0[L] & (fd[L] < f1[L]);
            eq[L] = in[L] & ((fd[L] == f0[L]) | ((NL > 1) & (fd[L] == f1[L])));
            any_eq |= eq[L];
        }
        if (__builtin_expect(__ballot(any_eq) != 0ull, 0)) {
#pragma unroll
            for (int L = 0; L < 3; ++L) {
                const int NL = L == 0 ? N0 : (L == 1 ? N1 : N2);
                if (eq[L]) {
                    const double e0 = p0k[L] >= 0 ? fabs((double)hu_s[p0k[L]] - m[L]) : INFINITY;
                    lt0[L] = before(hu_s, hidx_s, dd[L], uu[L], pp[L], e0, p0k[L]);
                    if (NL > 1) {
                        const double e1 = p1k[L] >= 0 ? fabs((double)hu_s[p1k[L]] - m[L]) : INFINITY;
                        lt1[L] = !lt0[L] && before(hu_s, hidx_s, dd[L], uu[L], pp[L], e1, p1k[L]);
                    }
                }
            }
        }
#pragma unroll
        for (int L = 0; L < 3; ++L) {
            const int NL = L == 0 ? N0 : (L == 1 ? N1 : N2);
            if (NL > 1) {   // lt0 and lt1 exclude each other
                f1[L] = lt1[L] ? fd[L] : f1[L];
                p1k[L] = lt1[L] ? pp[L] : p1k[L];
                f1[L] = lt0[L] ? f0[L] : f1[L];
                p1k[L] = lt0[L] ? p0k[L] : p1k[L];
            }
            f0[L] = lt0[L] ? fd[L] : f0[L];
            p0k[L] = lt0[L] ? pp[L] : p0k[L];
        }
    }
    // u of the kept hits, for the residuals
    float u0k[3], u1k[3];
#pragma unroll
    for (int L = 0; L < 3; ++L) {
        const int NL = L == 0 ? N0 : (L == 1 ? N1 : N2);
        u0k[L] = hu_s[p0k[L] >= 0 ? p0k[L] : p3];
        u1k[L] = NL > 1 ? hu_s[p1k[L] >= 0 ? p1k[L] : p3] : 0.0f;
    }
    int A[3][MAX_CLOSEST];
    int nA[3];
#pragma unroll
    for (int L = 0; L < 3; ++L) {
        A[L][0] = G.ncl[L] >= 1 ? p0k[L] : -1;
        A[L][1] = G.ncl[L] >= 2 ? p1k[L] : -1;
        nA[L] = (A[L][0] >= 0 ? 1 : 0) + (A[L][1] >= 0 ? 1 : 0);
    }
    // every option tuple of the item has the same layer set: a layer either
    // has hits (all its options are hits) or has the single option "no hit"
    const int mask = 8 | (nA[0] > 0 ? 1 : 0) | (nA[1] > 0 ? 2 : 0) | (nA[2] > 0 ? 4 : 0);
    const int n = __popc(mask);
    if (n < 3 || (mask & 3) == 0) return;
    if (DV1 && nA[0] == 0) return;   // the axial triplet needs its UTaX hit
    const FitConst fc = fit_const(G, mask);
    double r0[N0], r1[N1], r2[N2];
#pragma unroll
    for (int i = 0; i < N0; ++i) r0[i] = A[0][i] >= 0 ? (double)(i ? u1k[0] : u0k[0]) - sc.c[0] : 0.0;
#pragma unroll
    for (int i = 0; i < N1; ++i) r1[i] = A[1][i] >= 0 ? (double)(i ? u1k[1] : u0k[1]) - sc.c[1] : 0.0;
#pragma unroll
    for (int i = 0; i < N2; ++i) r2[i] = A[2][i] >= 0 ? (double)(i ? u1k[2] : u0k[2]) - sc.c[2] : 0.0;
    const int o0 = nA[0] > 0 ? nA[0] : 1, o1 = nA[1] > 0 ? nA[1] : 1, o2 = nA[2] > 0 ? nA[2] : 1;
#pragma unroll
    for (int i0 = 0; i0 < N0; ++i0) {
        if (i0 >= o0) continue;
#pragma unroll
        for (int i1 = 0; i1 < N1; ++i1) {
            if (i1 >= o1) continue;
#pragma unroll
            for (int i2 = 0; i2 < N2; ++i2) {
                if (i2 >= o2) continue;
                const double rho[4] = {r0[i0], r1[i1], r2[i2], rho3};
                double al, be, c2;
                fit_set(G, fc, rho, al, be, c2);
                const int bp[4] = {A[0][i0], A[1][i1], A[2][i2], p3};
                visit(n, ((cb * G.nw[0] + i0) * G.nw[1] + i1) * G.nw[2] + i2, al, be, c2, bp);
            }
        }
    }
}

// The paper's (1, 2, 2) closest hits are compiled on their own; other settings
// take the generic (<= 2, <= 2, <= 2) enumeration.  Same visiting order.
// cb: the UTbX hit's rank in its window (Dv0) or its index in its layer run (Dv1).
template <bool DV1 = false, typename Visit>
__device__ __forceinline__ void item_candidates(const DevGeom &G, const TrackArgs &a, const float *hu_s,
                                       const uint16_t *hidx_s, const uint16_t *E, const SeedConst &sc, int cb, int p3,
                                       Visit &&visit)
{
    if (G.ncl[0] == 1 && G.ncl[1] == 2 && G.ncl[2] == 2)
        item_candidates_n<1, 2, 2, DV1>(G, a, hu_s, hidx_s, E, sc, cb, p3, visit);
    else
        item_candidates_n<MAX_CLOSEST, MAX_CLOSEST, MAX_CLOSEST, DV1>(G, a, hu_s, hidx_s, E, sc, cb, p3, visit);
}

// Rank of the UTbX hit at p3 among the seed's first-window hits (by the
// window key), or -1 if it is outside the window.
__device__ __forceinline__ int first_window_rank(const DevGeom &G, const float *hu_s, const uint16_t *hidx_s,
                                        const SeedConst &sc, int p3)
{
    const double W1 = fma(G.w1c1, fabs((double)sc.q), G.w1c0);
    const double m3 = window1_centre(G, sc.c[3], (double)sc.q);
    const float u3 = hu_s[p3];
    const double d3 = fabs((double)u3 - m3);
    if (!(d3 <= W1)) return -1;
    const int i3 = hidx_s[p3];
    int rank = 0;
    // four positions per LDS round trip
    for (int p0 = sc.lo; p0 < sc.hi; p0 += 4) {
        float u[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) u[j] = hu_s[p0 + j < sc.hi ? p0 + j : p3];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int p = p0 + j;
            const double d = fabs((double)u[j] - m3);
            if (p < sc.hi && (d < d3 || (d == d3 && p != p3 && key_less(d, u[j], (int)hidx_s[p], d3, u3, i3)))) ++rank;
        }
    }
    return rank;
}

// Best candidate through one UTbX hit: more hits, then lower chi2, then lower index.
template <bool DV1 = false>
__device__ __forceinline__ void item_best(const DevGeom &G, const TrackArgs &a, const float *hu_s, const uint16_t *hidx_s,
                                 const uint16_t *E, const SeedConst &sc, int cb, int p3, int &best_n, double &best_chi2,
                                 int &best_c, int bp_out[4])
{
    best_n = 0;
    best_chi2 = 0.0;
    best_c = -1;
    item_candidates<DV1>(G, a, hu_s, hidx_s, E, sc, cb, p3,
                    [&](int n, int c, double, double, double c2, const int bp[4]) {
                        if (n > best_n || (n == best_n && c2 < best_chi2)) {
                            best_n = n;
                            best_chi2 = c2;
                            best_c = c;
#pragma unroll
                            for (int L = 0; L < 4; ++L) bp_out[L] = bp[L];
                        }
                    });
}

// The float32 track record of a fitted candidate; its ghost score is set by
// the caller (mlp_score_wave of the features, 0 without the network).
struct StoredTrack {
    float x, y, tx, ty, qop, chi2, score;
};

// A seed's float32 parameters.
struct SeedRaw {
    float x, y, tx, ty, qop;
};

__device__ __forceinline__ SeedRaw load_seed(const TrackArgs &a, int i)
{
    return SeedRaw{a.sx[i], a.sy[i], a.stx[i], a.sty[i], a.sqop[i]};
}

// f (optional): the track's ghost-killer features.
__device__ __forceinline__ StoredTrack stored_track(const DevGeom &G, const SeedRaw &sd, int n, double al, double be,
                                           double c2, const float *hu_s, const int bp[4], float *f)
{
    const float fsx = sd.x, fsy = sd.y, fstx = sd.tx, fsty = sd.ty, fsq = sd.qop;
    const double sx = fsx, sy = fsy, stx = fstx, sty = fsty;
    StoredTrack t;
    t.x = (float)(fma(stx, G.zref_seed, sx) + al);
    t.tx = (float)(stx + be);
    t.y = (float)fma(sty, G.zref_seed, sy);
    t.ty = fsty;
    t.qop = (G.mk != 0.0) ? (float)(-be / G.mk) : fsq;
    t.chi2 = (float)c2;
    t.score = 0.0f;
    if (f) {
        float hu4[4];
        int mask = 0;
#pragma unroll
        for (int L = 0; L < 4; ++L) {
            hu4[L] = bp[L] >= 0 ? hu_s[bp[L]] : 0.0f;
            mask |= bp[L] >= 0 ? (1 << L) : 0;
        }
        ghost_features(G, t.x, t.y, t.tx, t.ty, t.qop, t.chi2, n, fsx, fsy, fstx, fsty, fsq, hu4, mask, f);
    }
    return t;
}

// Write the selected candidate (LDS positions bp, -1 = none) as seed i's
// track, all but its ghost score; f (optional) receives its features.
__device__ __forceinline__ StoredTrack write_track(const TrackArgs &a, const DevGeom &G, int i, const SeedRaw &sd,
                                          const SeedConst &sc, const float *hu_s, const uint16_t *hidx_s, const int bp[4],
                                          int c, float *f)
{
    const int mask = (bp[0] >= 0 ? 1 : 0) | (bp[1] >= 0 ? 2 : 0) | (bp[2] >= 0 ? 4 : 0) | 8;
    const int n = __popc(mask);
    double rho[4];
#pragma unroll
    for (int L = 0; L < 4; ++L) rho[L] = bp[L] >= 0 ? (double)hu_s[bp[L]] - sc.c[L] : 0.0;
    double al, be, c2;
    fit_set(G, fit_const(G, mask), rho, al, be, c2);
    const StoredTrack t = stored_track(G, sd, n, al, be, c2, hu_s, bp, f);
    a.x[i] = t.x;
    a.y[i] = t.y;
    a.tx[i] = t.tx;
    a.ty[i] = t.ty;
    a.qop[i] = t.qop;
    a.chi2[i] = t.chi2;
    a.h0[i] = bp[0] >= 0 ? (int)hidx_s[bp[0]] : -1;
    a.h1[i] = bp[1] >= 0 ? (int)hidx_s[bp[1]] : -1;
    a.h2[i] = bp[2] >= 0 ? (int)hidx_s[bp[2]] : -1;
    a.h3[i] = (int)hidx_s[bp[3]];
    a.nhits[i] = n;
    if (a.cand) a.cand[i] = c;
    return t;
}

// One row per (seed, candidate index) of the candidate-scoring mode.
__device__ __forceinline__ void write_candidate_row(const TrackArgs &a, const DevGeom &G, int i, int n, int c, double al,
                                           double be, double c2, const float *hu_s, const uint16_t *hidx_s,
                                           const int bp[4])
{
    float f[NF];
    const StoredTrack t = stored_track(G, load_seed(a, i), n, al, be, c2, hu_s, bp, f);
    const size_t r = (size_t)i * (size_t)a.cmax + (size_t)c;
    a.r_seed[r] = i;
    a.r_cand[r] = c;
    a.r_nhits[r] = n;
    a.r_h0[r] = bp[0] >= 0 ? (int)hidx_s[bp[0]] : -1;
    a.r_h1[r] = bp[1] >= 0 ? (int)hidx_s[bp[1]] : -1;
    a.r_h2[r] = bp[2] >= 0 ? (int)hidx_s[bp[2]] : -1;
    a.r_h3[r] = (int)hidx_s[bp[3]];
    a.r_x[r] = t.x;
    a.r_y[r] = t.y;
    a.r_tx[r] = t.tx;
    a.r_ty[r] = t.ty;
    a.r_qop[r] = t.qop;
    a.r_chi2[r] = t.chi2;
    a.r_score[r] = mlp_score_lane(a.Wrow, f);
}

// The launch's binning parameters, read once per event and held in scalar
// registers (opaque to the compiler, which would otherwise re-load them from
// the argument segment, a scalar round trip, at every use).
struct BinParams {
    int nb, nbu, nb3, nbu3;
    float u0, inv_bw, inv_bw3;
};

template <typename T>
__device__ __forceinline__ T opaque_uniform(T v)
{
    asm volatile("" : "+s"(v));
    return v;
}

__device__ __forceinline__ BinParams bin_params(const TrackArgs &a)
{
    BinParams b;
    b.nb = opaque_uniform(a.nb);
    b.nbu = opaque_uniform(a.nbu);
    b.nb3 = opaque_uniform(a.nb3);
    b.nbu3 = opaque_uniform(a.nbu3);
    b.u0 = opaque_uniform(a.u0);
    b.inv_bw = opaque_uniform(a.inv_bw);
    b.inv_bw3 = opaque_uniform(a.inv_bw3);
    return b;
}

// Bucket of a hit: (layer, u bin) for Dv0; (layer, Y sector, u bin) for Dv1,
// with one last bucket per layer for sector ids outside [0, nsec).
template <bool DV1>
__device__ __forceinline__ int hit_bucket(const BinParams &bp, int nsec, int L, float u, int sec)
{
    const bool l3 = DV1 && L == 3;   // Dv0's layer 3 has the common layout
    const int nbu = l3 ? bp.nbu3 : bp.nbu;
    int b = L * bp.nb + bin_of(u, bp.u0, l3 ? bp.inv_bw3 : bp.inv_bw, nbu);
    if (DV1) b = sec < nsec ? b + sec * nbu : L * bp.nb + nsec * nbu;
    return b;
}

// The hits of one staging round of a layer (slot j: hit r 64 HPT + lane + 64 j
// of the run at `base`, n hits): their u and, for Dv1, their Y sector bytes,
// four to a word, loaded with them (not again at each use).
template <bool DV1, int HPT>
__device__ __forceinline__ void load_round(const TrackArgs &a, int base, int n, int r, float u[HPT],
                                           uint32_t sp[HPT / 4])
{
    // one lane pointer and constant offsets (64 j elements): no per-slot
    // address registers to keep; slot j is in the run iff lane < n - r 64 HPT - 64 j
    const int lane = threadIdx.x & 63;
    const int lim = n - r * 64 * HPT;
    const float *hp = a.hu + base + r * 64 * HPT + lane;
#pragma unroll
    for (int j = 0; j < HPT; ++j) u[j] = (lane < lim - 64 * j) ? hp[64 * j] : 0.0f;
    if (DV1) {
        const uint8_t *sp8 = a.hsec + base + r * 64 * HPT + lane;
#pragma unroll
        for (int q = 0; q < HPT / 4; ++q) sp[q] = 0u;
#pragma unroll
        for (int j = 0; j < HPT; ++j)
            if (lane < lim - 64 * j) sp[j >> 2] |= (uint32_t)sp8[64 * j] << (8 * (j & 3));
    }
}

template <int HPT>
__device__ __forceinline__ int slot_sector(const uint32_t sp[HPT / 4], int j)
{
    return (int)((sp[j >> 2] >> (8 * (j & 3))) & 0xffu);
}

constexpr int STAGE_HPT = 16;   // hits per lane per staging round

// Bucket bounds are 16-bit (an event's hits in LDS stay below 2^16): E[i] += 1
// through a 32-bit LDS atomic on the pair of bounds that holds it, returning
// the old E[i]; the low half never reaches 2^16, so it never carries into the
// high one.
__device__ __forceinline__ int bkt_add(uint16_t *E, int i)
{
    uint32_t *w = reinterpret_cast<uint32_t *>(E) + (i >> 1);
    const int sh = (i & 1) * 16;
    return (int)((atomicAdd(w, 1u << sh) >> sh) & 0xffffu);
}

// Zero the n 16-bit bounds at EL (one wavefront): 16-byte stores over the
// aligned middle, single bounds at the two ends.
__device__ __forceinline__ void zero_bounds(uint16_t *EL, int n)
{
    const int lane = threadIdx.x & 63;
    const int head = (int)((16 - (reinterpret_cast<uintptr_t>(EL) & 15)) & 15) / 2;   // bounds before 16-B alignment
    const int h = min(head, n);
    if (lane < h) EL[lane] = 0;
    const int nv = (n - h) / 8;   // whole 8-bound (16-byte) groups
    uint4 *V = reinterpret_cast<uint4 *>(EL + h);
    for (int q = lane; q < nv; q += 64) V[q] = make_uint4(0u, 0u, 0u, 0u);
    for (int b = h + 8 * nv + lane; b < n; b += 64) EL[b] = 0;
}

// Exclusive prefix, offset by `carry`, of the n 16-bit counts at EL (one
// wavefront), two counts per lane per step: a lane reads the pair (b, b + 1)
// of its 32-bit word, the wavefront sums the pairs (DPP, no LDS traffic) and
// the lane writes both starts back; eight independent 128-bound pieces per
// round, then the carries.  EL may start at an odd bound: the first and last
// bounds outside whole words go on their own.
__device__ __forceinline__ void scan_bounds(uint16_t *EL, int n, int carry)
{
    const int lane = threadIdx.x & 63;
    int first = 0;
    if (reinterpret_cast<uintptr_t>(EL) & 2) {   // EL[0] is the high half of a word
        first = n > 0 ? (int)EL[0] : 0;
        if (lane == 0 && n > 0) EL[0] = (uint16_t)carry;
        carry += first;
        ++EL;
        --n;
    }
    uint32_t *W = reinterpret_cast<uint32_t *>(EL);
    const int nw = n / 2;
    for (int w0 = 0; w0 < nw; w0 += 512) {
        uint32_t pr[8];
        int v[8], incl[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int w = w0 + 64 * j + lane;
            pr[j] = w < nw ? W[w] : 0u;
            v[j] = (int)(pr[j] & 0xffffu) + (int)(pr[j] >> 16);
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) incl[j] = wave_inclusive_sum(v[j]);
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int w = w0 + 64 * j + lane;
            const int s0 = carry + incl[j] - v[j], s1 = s0 + (int)(pr[j] & 0xffffu);
            if (w < nw) W[w] = (uint32_t)s0 | ((uint32_t)s1 << 16);
            carry += __builtin_amdgcn_readlane(incl[j], 63);
        }
    }
    if ((n & 1) && lane == 0) EL[n - 1] = (uint16_t)carry;   // a last bound in the low half of a word
}

// Stage one event's hits a wavefront per layer: each wavefront counts its
// layer's hits into the layer's buckets, scans them (two buckets per lane per
// step, DPP sums) and places the hits, with no workgroup barrier until the end: a
// wavefront's LDS operations complete in order.  Same result as a workgroup
// counting sort: E[b] = start of bucket b, E[3*nb + nb3] = count.  *s_bad must be 0
// on entry.
template <int BLOCK, bool DV1, typename Between>
__device__ __forceinline__ bool stage_hits_w(const TrackArgs &a, int nsec, int hb, const int hl[4], int nh,
                                             float *hu_s, uint16_t *hidx_s, uint16_t *E, int *s_bad, Between &&between)
{
    constexpr int HPT = STAGE_HPT;
    constexpr int NW = BLOCK / 64;
    // readfirstlane: the layer index is then known to be wavefront-uniform
    const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    // the first layer's loads are in flight while `between` runs
    int L = wave;
    int lo = L < 4 ? hl[L] : 0, n = L < 4 ? (L < 3 ? hl[L + 1] : nh) - hl[L] : 0;
    float u[HPT];
    uint32_t sp[HPT / 4];
    load_round<DV1, HPT>(a, hb + lo, n, 0, u, sp);
    if (tid == 0) E[0] = 0;
    between();
    const BinParams bp = bin_params(a);
    bool bad = false;
    for (; L < 4; L += NW) {
        if (L != wave) {   // a further layer of this wavefront (fewer than four wavefronts)
            lo = hl[L];
            n = (L < 3 ? hl[L + 1] : nh) - lo;
            load_round<DV1, HPT>(a, hb + lo, n, 0, u, sp);
        }
        uint16_t *EL = E + 1 + L * bp.nb;   // EL[b]: count, then end, of bucket (L, b)
        const int nb = (DV1 && L == 3) ? bp.nb3 : bp.nb;
        zero_bounds(EL, nb);
        const int rounds = (n + 64 * HPT - 1) / (64 * HPT);
        for (int r = 0; r < rounds; ++r) {
            if (r > 0) load_round<DV1, HPT>(a, hb + lo, n, r, u, sp);
#pragma unroll
            for (int j = 0; j < HPT; ++j) {
                if (r * 64 * HPT + 64 * j >= n) break;   // uniform: no lane has slot j
                const int k = r * 64 * HPT + lane + 64 * j;
                if (k < n) {
                    if (!isfinite(u[j])) bad = true;
                    else bkt_add(E, hit_bucket<DV1>(bp, nsec, L, u[j], slot_sector<HPT>(sp, j)) + 1);
                }
            }
        }
        scan_bounds(EL, nb, lo);
        // placing pass: EL[b] advances to the end of bucket b
        for (int r = 0; r < rounds; ++r) {
            if (rounds > 1) load_round<DV1, HPT>(a, hb + lo, n, r, u, sp);
#pragma unroll
            for (int j = 0; j < HPT; ++j) {
                if (r * 64 * HPT + 64 * j >= n) break;
                const int k = r * 64 * HPT + lane + 64 * j;
                if (k < n && isfinite(u[j])) {
                    const int pos = bkt_add(E, hit_bucket<DV1>(bp, nsec, L, u[j], slot_sector<HPT>(sp, j)) + 1);
                    hu_s[pos] = u[j];
                    hidx_s[pos] = (uint16_t)k;
                }
            }
        }
    }
    if (bad) *s_bad = 1;
    lds_barrier();
    return *s_bad == 0;
}

__device__ __forceinline__ bool pca64(const DevGeom &G, double x1, double y1, double tx1, double ty1, double g1, double x2,
                             double y2, double tx2, double ty2, double g2, double &vx, double &vy, double &vz,
                             double &doca, double &s_out, double &t_out);
__device__ __forceinline__ void vertex_extras(const DevGeom &G, const float *WLg, float4 A, float4 B, double g1, double g2,
                                     float q1, float q2, double s, double t, float4 V, float out[6]);

// Vertexing of one event by the whole workgroup.  Only opposite-charge pairs
// are visited: the kept tracks sit in LDS split by seed charge (Kept below),
// and row r of the pair triangle (the r-th kept track in slot order) holds its
// opposite-charge partners of higher slot, which are a run of the other charge
// list; rows are concatenated in slot order, so pair ranks follow (i, j)
// order.  Each lane takes VTX_PPT consecutive pairs of a chunk (a binary
// search of the row starts, then steps along the row) and applies the float32
// straight-line prescreen; the chunk's survivors are appended, in pair order,
// to a ring of pair codes in LDS (one workgroup scan per chunk).  Whenever a
// workgroup's worth of survivors is queued (and at the end) they are fitted
// together, a lane per pair (float64 Newton PCA), and the passing ones
// written in queue order: vertices come out (i, j)-ordered, and the first vcap
// of them are kept.  ring: vtx_ring<BLOCK>() ints.  XTR: also the masses and
// trigger-line scores of each vertex (compiled only where they are asked for:
// their registers would otherwise count against every fused launch).
// VTX_PPT = 5: neighbouring lanes read partners 5 entries (80 bytes) apart,
// which spreads a wavefront's 16-byte LDS reads over distinct banks.
constexpr int VTX_PPT = 5;
__host__ __device__ constexpr int vtx_ring_ints(int block)   // a power of two above the block - 1 + VTX_PPT * block live entries
{
    int r = 1;
    while (r < (VTX_PPT + 1) * block) r *= 2;
    return r;
}
template <int BLOCK>
constexpr int vtx_ring() { return vtx_ring_ints(BLOCK); }

// Kept tracks of one event in LDS, the vertexing input.  Positive-charge
// tracks fill st/q/slot from the front and negative ones from the back, each
// list in slot order (the o-th negative at tcap - 1 - o).  The vertexing
// derives the row table from them: row[r] describes the r-th kept track in
// slot order (its index o in its charge list, | 0x8000 when positive; the
// tracks of the other charge before it number r - o, so its partners of
// higher slot are that list's entries from r - o on), and R[r] is the rank of
// row r's first pair (R[n] = all pairs).  The table lives apart from the list
// (in the fused kernel, on buffers that are dead by then).
struct Kept {
    float4 *st;      // x, y, tx, ty at the UT midpoint
    float *q;        // fitted q/p
    int *slot;       // slot << 1 | positive seed charge
    int *R;          // tcap + 1 row starts
    uint16_t *row;   // tcap row descriptors
};

__host__ __device__ constexpr size_t kept_lds_bytes(int tcap)
{
    return tcap > 0 ? ((size_t)tcap * 24 + 15) & ~(size_t)15 : 0;
}

__host__ __device__ constexpr size_t kept_rows_bytes(int tcap)
{
    return tcap > 0 ? ((size_t)tcap * 6 + 4 + 15) & ~(size_t)15 : 0;
}

__device__ __forceinline__ Kept kept_carve(unsigned char *base, unsigned char *rows, int tcap)
{
    Kept k;
    k.st = reinterpret_cast<float4 *>(base);
    k.q = reinterpret_cast<float *>(base + (size_t)tcap * 16);
    k.slot = reinterpret_cast<int *>(base + (size_t)tcap * 20);
    k.R = reinterpret_cast<int *>(rows);
    k.row = reinterpret_cast<uint16_t *>(rows + (size_t)tcap * 4 + 4);
    return k;
}

// Appends this chunk's kept tracks (at most one per lane, lanes in slot
// order).  n and np (kept so far, positive so far) are workgroup-uniform and
// advanced; tcap < 32768 (LDS holds far fewer).
template <int BLOCK>
__device__ __forceinline__ void kept_append(const Kept &K, int tcap, bool kept, bool positive, float4 st, float q,
                                            int slot, int &n, int &np, int *s_wsum)
{
    int tot;
    const int ex = block_exclusive_scan<BLOCK>(kept ? (positive ? 0x10001 : 1) : 0, s_wsum, &tot);
    if (kept) {
        const int r = n + (ex & 0xffff);
        const int pb = np + (ex >> 16);   // positive tracks before this one
        const int pos = positive ? pb : tcap - 1 - (r - pb);
        K.st[pos] = st;
        K.q[pos] = q;
        K.slot[pos] = (slot << 1) | (positive ? 1 : 0);
    }
    n += tot & 0xffff;
    np += tot >> 16;
}

// Number of entries of a charge list (m of them, slot order) with a slot
// below sl: the list's i-th slot is at K.slot[b + d * i].
__device__ __forceinline__ int slots_below(const Kept &K, int b, int d, int m, int sl)
{
    int lo = 0;
    for (int step = m > 0 ? 1 << (31 - __builtin_clz(m)) : 0; step > 0; step >>= 1)
        if (lo + step <= m && (K.slot[b + d * (lo + step - 1)] >> 1) < sl) lo += step;
    return lo;
}

__device__ __forceinline__ bool pair_prescreen(const DevGeom &G, float4 A, float4 B)
{
    const float wx = A.x - B.x, wy = A.y - B.y;
    const float nx = A.w - B.w, ny = B.z - A.z;
    const float nz = fmaf(A.z, B.w, -(A.w * B.z));
    const float wn = fmaf(wx, nx, wy * ny);
    const float nn = fmaf(nx, nx, fmaf(ny, ny, nz * nz));
    return (nn < 1e-6f) || (wn * wn < G.prescreen_thr2 * nn);
}

// Args: TrackArgs (fused step) or VertexArgs (standalone): the vertex outputs
// vcap, vcount, vi, vj, vx, vy, vz, vdoca, voverflow, the extras' outputs, WL
// and the seeds' sqop under the same names.  n kept tracks, np of them
// positive, in K (kept_append); the row list is visible to every lane.
template <int BLOCK, bool XTR, typename Args>
__device__ __forceinline__ void vertex_event_block(const Args &a, const DevGeom &G, int e, int s0, int n, int np,
                                          const Kept &K, int tcap, int *ring, int *s_wsum)
{
    constexpr int CH = VTX_PPT * BLOCK, RING = vtx_ring<BLOCK>();
    static_assert((RING & (RING - 1)) == 0, "ring size a power of two");
    const int tid = threadIdx.x;
    const bool curved = (G.fp != 0.0);
    const int nn = n - np;   // negative tracks
    // row table: each track's rank in slot order (its index in its list plus
    // the tracks of the other list with a lower slot), then the row starts;
    // row r pairs with the other list's entries from r - o on
    int npairs = 0;
    if (np > 0 && nn > 0) {
        for (int e0 = 0; e0 < n; e0 += BLOCK) {
            const int e = e0 + tid;
            if (e < n) {
                const bool pos = e < np;
                const int o = pos ? e : e - np;
                const int sl = K.slot[pos ? o : tcap - 1 - o] >> 1;
                const int r = o + (pos ? slots_below(K, tcap - 1, -1, nn, sl) : slots_below(K, 0, 1, np, sl));
                K.row[r] = (uint16_t)(o | (pos ? 0x8000 : 0));
            }
        }
        lds_barrier();
        for (int r0 = 0; r0 < n; r0 += BLOCK) {
            const int r = r0 + tid;
            int len = 0;
            if (r < n) {
                const int d = K.row[r];
                len = ((d & 0x8000) ? nn : np) - (r - (d & 0x7fff));
            }
            int tot;
            const int ex = block_exclusive_scan<BLOCK>(len, s_wsum, &tot);
            if (r < n) K.R[r] = npairs + ex;
            npairs += tot;
        }
        if (tid == 0) K.R[n] = npairs;
        lds_barrier();
    }
    const int top = n > 1 ? 1 << (31 - __builtin_clz(n - 1)) : 0;   // highest power of two below n
    int out_n = 0, head = 0, qn = 0;   // workgroup-uniform
    for (int chunk = 0;;) {
        const bool more = chunk < npairs;
        if (more) {
            const int k0 = chunk + VTX_PPT * tid;
            int code[VTX_PPT];
            unsigned m = 0;
            if (k0 < npairs) {
                // row of k0: the last r with R[r] <= k0 (a row without pairs starts where the next one does)
                int r = 0;
                for (int step = top; step > 0; step >>= 1)
                    if (r + step < n && K.R[r + step] <= k0) r += step;
                int rend = K.R[r + 1], c = k0 - K.R[r];
                int d = K.row[r];
                int pa = (d & 0x8000) ? (d & 0x7fff) : tcap - 1 - (d & 0x7fff);
                float4 A = K.st[pa];
                int k = k0;
#pragma unroll
                for (int j = 0; j < VTX_PPT; ++j) {
                    if (j > 0) {
                        ++k;
                        ++c;
                        if (k >= rend && k < npairs) {   // on to the next row that has pairs
                            do {
                                ++r;
                            } while (K.R[r + 1] <= k);
                            rend = K.R[r + 1];
                            c = k - K.R[r];
                            d = K.row[r];
                            pa = (d & 0x8000) ? (d & 0x7fff) : tcap - 1 - (d & 0x7fff);
                            A = K.st[pa];
                        }
                    }
                    // past the last pair nothing is read out of range; the prescreen runs on every lane
                    const bool valid = k < npairs;
                    const int q = r - (d & 0x7fff) + c;   // partner index in the other list
                    const int pb = valid ? ((d & 0x8000) ? tcap - 1 - q : q) : pa;
                    code[j] = (pa << 16) | pb;
                    const bool near = curved | pair_prescreen(G, A, K.st[pb]);
                    m |= (valid & near) ? 1u << j : 0u;
                }
            }
            int tot;
            int pos = block_exclusive_scan<BLOCK>(__popc(m), s_wsum, &tot);
#pragma unroll
            for (int j = 0; j < VTX_PPT; ++j)
                if ((m >> j) & 1u) ring[(head + qn + pos++) & (RING - 1)] = code[j];
            qn += tot;
            chunk += CH;
        }
        // fit the queued survivors a workgroup at a time (all of them at the end)
        while (qn >= BLOCK || (!more && qn > 0)) {
            lds_barrier();   // the queued codes are visible
            const int take = min(qn, BLOCK);
            int pass = 0, ia = 0, ib = 0;
            float4 R;
            float2 ST;
            if (tid < take) {
                const int c = ring[(head + tid) & (RING - 1)];
                ia = c >> 16;
                ib = c & 0xffff;
                const float4 A = K.st[ia], B = K.st[ib];
                const double g1 = -G.fp * (G.gc0 + G.gc1 * ((double)K.q[ia] * 1e-3));
                const double g2 = -G.fp * (G.gc0 + G.gc1 * ((double)K.q[ib] * 1e-3));
                double vx, vy, vz, dd, ps, pt;
                const bool good = pca64(G, A.x, A.y, A.z, A.w, g1, B.x, B.y, B.z, B.w, g2, vx, vy, vz, dd, ps, pt);
                pass = (good && (dd < G.doca_max)) ? 1 : 0;
                R = make_float4((float)vx, (float)vy, (float)vz, (float)dd);
                ST = make_float2((float)ps, (float)pt);
            }
            int tot2;
            const int opos = block_exclusive_scan<BLOCK>(pass, s_wsum, &tot2);
            if (pass) {
                const int m2 = out_n + opos;
                if (m2 < a.vcap) {
                    const size_t o = (size_t)e * (size_t)a.vcap + (size_t)m2;
                    a.vi[o] = K.slot[ia] >> 1;
                    a.vj[o] = K.slot[ib] >> 1;
                    a.vx[o] = R.x;
                    a.vy[o] = R.y;
                    a.vz[o] = R.z;
                    a.vdoca[o] = R.w;
                    if constexpr (XTR) {
                        const float4 TA = K.st[ia], TB = K.st[ib];
                        const double g1 = -G.fp * (G.gc0 + G.gc1 * ((double)K.q[ia] * 1e-3));
                        const double g2 = -G.fp * (G.gc0 + G.gc1 * ((double)K.q[ib] * 1e-3));
                        float ex[6];
                        vertex_extras(G, a.WL, TA, TB, g1, g2, a.sqop[s0 + (K.slot[ia] >> 1)],
                                      a.sqop[s0 + (K.slot[ib] >> 1)], ST.x, ST.y, R, ex);
                        a.m_pipi[o] = ex[0];
                        a.m_ppi[o] = ex[1];
                        a.line0[o] = ex[2];
                        a.line1[o] = ex[3];
                        a.line2[o] = ex[4];
                        a.line3[o] = ex[5];
                    }
                }
            }
            out_n += tot2;
            head += take;
            qn -= take;
        }
        if (!more) break;
    }
    if (tid == 0) {
        a.vcount[e] = out_n < a.vcap ? out_n : a.vcap;
        if (out_n > a.vcap) atomicAdd(a.voverflow, out_n - a.vcap);
    }
}

// Event of launch iteration `iter`: the work counter of a persistent launch,
// or the one event of a per-event launch.
__device__ __forceinline__ int grab_event(const TrackArgs &a, int iter)
{
    if (a.ev_single >= 0) return iter == 0 ? a.ev_single : a.n_events;
    const int k = atomicAdd(&a.counter[0], 1);
    return (a.order && k < a.n_events) ? a.order[k] : k;
}

// One whole wave: the event of iteration `iter` and its offsets into LDS,
// s_nx = {event, seed_off[e], seed_off[e + 1], hit_off[4e .. 4e + 4]}.
__device__ __forceinline__ void fetch_event(const TrackArgs &a, int iter, int lane, int *s_nx)
{
    int en = 0;
    if (lane == 0) en = grab_event(a, iter);
    en = __builtin_amdgcn_readfirstlane(en);
    if (lane == 0) s_nx[0] = en;
    if (lane < 7 && en < a.n_events) s_nx[1 + lane] = lane < 2 ? a.seed_off[en + lane] : a.hit_off[4 * en + lane - 2];
}

// XTR (with VTX): the fused vertexing also writes masses and trigger-line scores.
template <int BLOCK, bool CANDS, bool VTX, bool DV1, bool XTR = false>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(CANDS ? 2 : 3))) void k_track(TrackKernArgs)
{
    static_assert(!(CANDS && DV1), "candidate rows follow Dv0");
    static_assert(!XTR || VTX, "extras come with the fused vertexing");
    const TrackArgs &a0 = kernel_args<TrackKernArgs>().a;
    extern __shared__ __align__(16) unsigned char smem[];
    size_t off = 0;
    float *hu_s = reinterpret_cast<float *>(smem + off);
    off += (size_t)a0.hcap * 4;
    uint16_t *hidx_s = reinterpret_cast<uint16_t *>(smem + off);
    off = (off + (size_t)a0.hcap * 2 + 15) & ~(size_t)15;
    uint16_t *E = reinterpret_cast<uint16_t *>(smem + off);
    off = (off + (size_t)(3 * a0.nb + a0.nb3 + 1) * 2 + 15) & ~(size_t)15;
    SeedConst *s_c = reinterpret_cast<SeedConst *>(smem + off);
    off += (size_t)BLOCK * sizeof(SeedConst);
    unsigned long long *s_key = reinterpret_cast<unsigned long long *>(smem + off);
    off += (size_t)BLOCK * 8;
    int *s_base = reinterpret_cast<int *>(smem + off);
    off = (off + (size_t)BLOCK * 4 + 15) & ~(size_t)15;
    uint32_t *it_desc = reinterpret_cast<uint32_t *>(smem + off);
    off = (off + (size_t)a0.icap * 4 + 15) & ~(size_t)15;
    unsigned long long *it_hits = reinterpret_cast<unsigned long long *>(smem + off);
    off = (off + (size_t)a0.icap * 8 + 15) & ~(size_t)15;
    // fused vertexing: kept tracks of the event (its survivor ring aliases the seed constants);
    // the list's pointers are derived where they are used
    const uint32_t kept_off = (uint32_t)off;
    __shared__ int s_nx[8];   // next event and its offsets (fetch_event)
    __shared__ int s_bad, s_nacc, s_nitems, s_nkept, s_nkpos;
    __shared__ int s_long;   // Dv1: a seed of the chunk has more than 128 UTbX hits
    __shared__ int s_wsum[BLOCK / 64];
    const int tid = threadIdx.x;

    // The next event is fetched while this one is processed: its index (the
    // work counter's atomic) and offsets arrive during phase B, where the
    // last wave, the one with the fewest items, waits for them.
    if (tid < 64) fetch_event(a0, 0, tid, s_nx);
    lds_barrier();
    for (int iter = 0;; ++iter) {
        const TrackKernArgs &Ke = kernel_args<TrackKernArgs>();
        const TrackArgs &a = Ke.a;
        const DevGeom &G = Ke.G;
        const int e = s_nx[0];
        if (e >= a.n_events) break;
        const int s0 = s_nx[1], s1 = s_nx[2];
        int ho[5];
#pragma unroll
        for (int L = 0; L < 5; ++L) ho[L] = s_nx[3 + L];
        if (tid == 0) s_bad = 0;
        lds_barrier();   // s_nx read by every wave before it is refilled
        const bool seeds_ok = (0 <= s0) && (s0 <= s1) && (s1 <= a.n_seeds);
        bool hits_ok = (0 <= ho[0]) && (ho[4] <= a.n_hits);
#pragma unroll
        for (int L = 0; L < 4; ++L) hits_ok = hits_ok && (ho[L] <= ho[L + 1]) && (ho[L + 1] - ho[L] <= 65535);
        const int nh = ho[4] - ho[0];
        int bad = 0;
        if (!seeds_ok || !hits_ok) bad = F_BAD_OFFSETS;
        else if (nh > a.hcap || nh > a.max_hits || s1 - s0 > a.max_seeds) bad = F_CAPACITY;
        if (bad) {
            if (tid == 0) atomicOr(a.flags, bad);
            if (VTX && tid == 0) a.vcount[e] = 0;
            if (seeds_ok)
                for (int i = s0 + tid; i < s1; i += BLOCK) write_empty_track(a, i);
            if (tid < 64) fetch_event(a, iter + 1, tid, s_nx);
            lds_barrier();
            continue;
        }
        if (s1 == s0) {
            if (VTX && tid == 0) a.vcount[e] = 0;
            if (tid < 64) fetch_event(a, iter + 1, tid, s_nx);
            lds_barrier();
            continue;
        }
        if (VTX && tid == 0) s_nkept = s_nkpos = 0;
        int hl[4];
#pragma unroll
        for (int L = 0; L < 4; ++L) hl[L] = ho[L] - ho[0];
        // seed frames of the first chunk, computed while the hits are loading;
        // the seeds are loaded first, so that the frames wait for them alone
        const bool have0 = tid < s1 - s0;
        SeedRaw sd0{};
        if (have0) sd0 = load_seed(a, s0 + tid);
        auto first_frames = [&]() {
            if (have0) {
                SeedConst sc;
                double m3, W1;
                if (!seed_frame(G, sd0.x, sd0.y, sd0.tx, sd0.ty, sd0.qop, sc, m3, W1)) {
                    atomicOr(a.flags, F_NONFINITE);
                    sc.q = __int_as_float(0x7fc00000);   // NaN: no frame
                } else if (DV1) {
                    seed_sectors(G, sd0.y, sd0.ty, sc);
                }
                s_c[tid] = sc;
            }
        };
        if (!stage_hits_w<BLOCK, DV1>(a, G.nsec, ho[0], hl, nh, hu_s, hidx_s, E, &s_bad, first_frames)) {
            if (tid == 0) atomicOr(a.flags, F_NONFINITE);
            if (VTX && tid == 0) a.vcount[e] = 0;
            for (int i = s0 + tid; i < s1; i += BLOCK) write_empty_track(a, i);
            if (tid < 64) fetch_event(a, iter + 1, tid, s_nx);
            lds_barrier();
            continue;
        }

        // seeds in chunks of at most BLOCK, shortened so that their items fit
        for (int sc0 = s0; sc0 < s1;) {
            const TrackKernArgs &Kc = kernel_args<TrackKernArgs>();
            const TrackArgs &a = Kc.a;
            const DevGeom &G = Kc.G;
            if (tid == 0) {
                s_nacc = min(BLOCK, s1 - sc0);
                s_nitems = INT_MAX;
                s_long = 0;
            }
            // phase A: lane per seed, the UTbX bucket range of its first window;
            // every hit of the range inside the window becomes an item (seed, hit)
            const int i = sc0 + tid;
            const bool have = i < s1;
            SeedConst sc;
            double m3 = 0.0, W1 = 0.0;
            int n_rng = 0, p_lo = 0, p_hi = 0;
            if (have) {
                bool ok;
                if (sc0 == s0) {
                    sc = s_c[tid];
                    ok = sc.q == sc.q;
                    m3 = window1_centre(G, sc.c[3], (double)sc.q);
                    W1 = fma(G.w1c1, fabs((double)sc.q), G.w1c0);
                } else {
                    ok = seed_frame(G, a.sx[i], a.sy[i], a.stx[i], a.sty[i], a.sqop[i], sc, m3, W1);
                    if (!ok) atomicOr(a.flags, F_NONFINITE);
                    else if (DV1) seed_sectors(G, a.sy[i], a.sty[i], sc);
                }
                if (ok) {
                    if (DV1) {
                        // Dv1: every UTbX hit of the compatible sectors, no momentum window
                        int klo, khi;
                        sector_span(sc, 3, klo, khi);
                        if (klo <= khi) {
                            p_lo = E[3 * a.nb + klo * a.nbu3];
                            p_hi = E[3 * a.nb + (khi + 1) * a.nbu3];
                        }
                    } else if (G.max_l3 > 0) {
                        bin_range(E, 3, a.nb, a.u0, a.inv_bw, m3, W1, p_lo, p_hi);
                    }
                    n_rng = p_hi - p_lo;
                }
            }
            if (!DV1) {   // Dv1 keeps its sector spans in lo / hi
                sc.lo = (uint16_t)p_lo;
                sc.hi = (uint16_t)p_hi;
            }
            // an item per UTbX hit inside the first window (Dv0) or per axial triplet (Dv1)
            const double W2 = DV1 ? fma(G.w2c1, fabs((double)sc.q), G.w2c0) : 0.0;
            int k0lo = 0, k0hi = -1;
            if (DV1) sector_span(sc, 0, k0lo, k0hi);
            auto is_item = [&](int p) {
                return DV1 ? dv1_triplet(G, a, hu_s, E, sc, k0lo, k0hi, W2, p) : fabs((double)hu_s[p] - m3) <= W1;
            };
            int n_win = 0;
            uint32_t in_mask = 0;   // Dv0: in-window flags of the range's first 32 hits
            // Dv1 tests its axial triplets a wavefront per seed, a lane per UTbX
            // hit (tens of hits per seed): the seed constants and ranges go to LDS
            int *s_pk = reinterpret_cast<int *>(it_hits);   // free until phase B
            int *s_cnt = reinterpret_cast<int *>(s_key);    // free until the scan below
            // triplet flags of a seed's first 128 UTbX hits, kept for the write pass
            unsigned long long *s_mask = it_hits + BLOCK / 2;
            // readfirstlane: the compiler then knows the wavefront index is uniform
            const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
            const int n_chunk = min(BLOCK, s1 - sc0);
            if (DV1) {
                s_c[tid] = sc;
                s_pk[tid] = p_lo | (n_rng << 16);
                lds_barrier();
                // two seeds per pass, so that their LDS round trips overlap; a lane
                // past a seed's range probes hit 0 (in bounds) and is masked off
                for (int sl = wave; sl < n_chunk; sl += 2 * (BLOCK / 64)) {
                    const int sl2 = sl + BLOCK / 64;
                    const bool two = sl2 < n_chunk;
                    const int pk = s_pk[sl], pk2 = two ? s_pk[sl2] : 0;
                    const int plo = pk & 0xffff, nr = pk >> 16, plo2 = pk2 & 0xffff, nr2 = pk2 >> 16;
                    const SeedConst scw = s_c[sl], scw2 = s_c[two ? sl2 : sl];
                    const double W2w = fma(G.w2c1, fabs((double)scw.q), G.w2c0);
                    const double W2w2 = fma(G.w2c1, fabs((double)scw2.q), G.w2c0);
                    int klo, khi, klo2, khi2;
                    sector_span(scw, 0, klo, khi);
                    sector_span(scw2, 0, klo2, khi2);
                    int cnt = 0, cnt2 = 0;
                    for (int k0 = 0; k0 < max(nr, nr2); k0 += 64) {
                        const int k = k0 + lane;
                        const bool v1 = k < nr, v2 = k < nr2;
                        TripletProbe t1, t2;
                        dv1_probe_pair(G, a, hu_s, E, scw, scw2, klo, khi, klo2, khi2, W2w, W2w2, v1 ? plo + k : 0,
                                       v2 ? plo2 + k : 0, t1, t2);
                        // ballots of both first probes on every lane (nothing to sink into a
                        // branch), the rare longer windows after them
                        const unsigned long long h1 = __ballot(t1.hit), h2 = __ballot(t2.hit);
                        const bool r1 = v1 && !t1.hit && dv1_rest(hu_s, t1, W2w, DV1_PROBE);
                        const bool r2 = v2 && !t2.hit && dv1_rest(hu_s, t2, W2w2, DV1_PROBE);
                        const unsigned long long m = (h1 & __ballot(v1)) | __ballot(r1);
                        const unsigned long long m2 = (h2 & __ballot(v2)) | __ballot(r2);
                        if (k0 < 128 && lane == 0) {
                            s_mask[2 * sl + (k0 >> 6)] = m;
                            if (two) s_mask[2 * sl2 + (k0 >> 6)] = m2;
                        }
                        cnt += __popcll(m);
                        cnt2 += __popcll(m2);
                    }
                    if (lane == 0) {
                        s_cnt[sl] = cnt;
                        if (two) s_cnt[sl2] = cnt2;
                        if (max(nr, nr2) > 128) s_long = 1;
                    }
                }
                lds_barrier();
                n_win = have ? s_cnt[tid] : 0;
            } else {
                // four positions per LDS round trip
                for (int k0 = 0; k0 < n_rng; k0 += 4) {
                    float u[4];
#pragma unroll
                    for (int j = 0; j < 4; ++j) u[j] = hu_s[k0 + j < n_rng ? p_lo + k0 + j : p_lo];
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int k = k0 + j;
                        const bool in = k < n_rng && fabs((double)u[j] - m3) <= W1;
                        n_win += in ? 1 : 0;
                        in_mask |= (in && k < 32) ? 1u << k : 0u;
                    }
                }
            }
            int tot;
            const int excl = block_exclusive_scan<BLOCK>(n_win, s_wsum, &tot);
            bool acc = have && (excl + n_win <= a.icap);
            if (tid == 0 && have && !acc) {
                // one seed alone overflows the item buffer: keep its first items (flagged)
                atomicOr(a.flags, F_CAPACITY);
                n_win = a.icap;
                acc = true;
            }
            // acceptance is a prefix of the chunk; only the (rare) refused seeds
            // touch the shared counters: the first refused one ends the chunk
            // and its exclusive offset is the chunk's item count
            if (have && !acc) {
                atomicMin(&s_nacc, tid);
                atomicMin(&s_nitems, excl);
            }
            if (acc) {
                s_c[tid] = sc;
                s_key[tid] = ~0ull;
                s_base[tid] = excl;
                if (!DV1) {
                    if (n_rng <= 32) {
                        uint32_t m = in_mask;
                        for (int w = 0; m != 0 && w < n_win; ++w) {
                            const int k = __ffs(m) - 1;
                            m &= m - 1;
                            it_desc[excl + w] = ((uint32_t)tid << 16) | (uint32_t)(p_lo + k);
                        }
                    } else {
                        for (int k = 0, w = 0; k < n_rng && w < n_win; ++k) {
                            if (is_item(p_lo + k)) it_desc[excl + w++] = ((uint32_t)tid << 16) | (uint32_t)(p_lo + k);
                        }
                    }
                } else {
                    // Dv1, lane per seed: the triplets among the first 128 UTbX hits,
                    // from the counting pass's flags, in hit order
                    int w = 0;
#pragma unroll
                    for (int j = 0; j < 2; ++j) {
                        unsigned long long m = 64 * j < n_rng ? s_mask[2 * tid + j] : 0ull;
                        for (; m != 0 && w < n_win; ++w) {
                            const int k = 64 * j + __ffsll((long long)m) - 1;
                            m &= m - 1;
                            it_desc[excl + w] = ((uint32_t)tid << 16) | (uint32_t)(p_lo + k);
                        }
                    }
                }
            }
            if (DV1 && __builtin_amdgcn_readfirstlane(s_long)) {   // uniform: written before a barrier
                // seeds with more than 128 UTbX hits: the rest of their triplets, a
                // wavefront per seed, after the flagged ones
                lds_barrier();
                const int nacc_w = s_nacc, nit_w = min(min(tot, s_nitems), a.icap);
                for (int sl = wave; sl < nacc_w; sl += BLOCK / 64) {
                    const int pk = s_pk[sl], plo = pk & 0xffff, nr = pk >> 16;
                    if (nr <= 128) continue;
                    const SeedConst scw = s_c[sl];
                    const double W2w = fma(G.w2c1, fabs((double)scw.q), G.w2c0);
                    int klo, khi;
                    sector_span(scw, 0, klo, khi);
                    const int base = s_base[sl], cap = (sl + 1 < nacc_w ? s_base[sl + 1] : nit_w) - base;
                    int w = __popcll(s_mask[2 * sl]) + __popcll(s_mask[2 * sl + 1]);
                    for (int k0 = 128; k0 < nr && w < cap; k0 += 64) {
                        const bool f = k0 + lane < nr && dv1_triplet(G, a, hu_s, E, scw, klo, khi, W2w, plo + k0 + lane);
                        const unsigned long long m = __ballot(f);
                        const int pre = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32),
                                                                   __builtin_amdgcn_mbcnt_lo((unsigned)m, 0));
                        if (f && w + pre < cap)
                            it_desc[base + w + pre] = ((uint32_t)sl << 16) | (uint32_t)(plo + k0 + lane);
                        w += __popcll(m);
                    }
                }
            }
            lds_barrier();
            const int nacc = s_nacc, n_items = min(min(tot, s_nitems), a.icap);
            if (sc0 == s0 && tid >= BLOCK - 64) fetch_event(a, iter + 1, tid - (BLOCK - 64), s_nx);
            // phase B: lane per (seed, UTbX hit) item
            for (int it = tid; it < n_items; it += BLOCK) {
                const TrackKernArgs &Ki = kernel_args<TrackKernArgs>();
                const TrackArgs &a = Ki.a;
                const DevGeom &G = Ki.G;
                const uint32_t d = it_desc[it];
                const int sl = (int)(d >> 16), p3 = (int)(d & 0xffffu);
                const SeedConst scs = s_c[sl];
                int r3;
                if (DV1) {
                    r3 = hidx_s[p3];   // Dv1 candidate index: the UTbX hit's index in its run
                } else {
                    const int base = s_base[sl];
                    const int nwin = (sl + 1 < nacc ? s_base[sl + 1] : n_items) - base;
                    if (CANDS || nwin > G.max_l3) {
                        r3 = first_window_rank(G, hu_s, hidx_s, scs, p3);
                        if (r3 < 0 || r3 >= G.max_l3) continue;
                    } else {
                        // every window hit is kept: the item's position stands in for its
                        // rank (it orders only exact ties); phase C ranks the winner
                        r3 = it - base;
                    }
                }
                if (CANDS) {
                    item_candidates(G, a, hu_s, hidx_s, E, scs, r3, p3,
                                    [&](int n, int c, double al, double be, double c2, const int bp[4]) {
                                        write_candidate_row(a, G, sc0 + sl, n, c, al, be, c2, hu_s, hidx_s, bp);
                                    });
                    continue;
                }
                int bn, bc, bp[4] = {-1, -1, -1, -1};
                double bchi2;
                item_best<DV1>(G, a, hu_s, hidx_s, E, scs, r3, p3, bn, bchi2, bc, bp);
                if (bn > 0) {
                    unsigned long long packed = 0;
#pragma unroll
                    for (int L = 0; L < 4; ++L)
                        packed |= (unsigned long long)(bp[L] >= 0 ? (unsigned)bp[L] : 0xffffu) << (16 * L);
                    it_hits[DV1 ? it : s_base[sl] + r3] = packed;
                    atomicMin(&s_key[sl], DV1 ? pack_key_dv1(bn, bchi2, bc) : pack_key(bn, bchi2, bc));
                }
            }
            // the seed parameters of phase C are loaded before the barrier: their
            // latency overlaps the wait
            SeedRaw sd{};
            if (!CANDS && tid < nacc) sd = load_seed(a, i);
            lds_barrier();
            // phase C: lane per seed, write the winner; then its ghost score, the
            // network run by each wavefront with a winner as a whole
            bool won = false;
            StoredTrack t;
            int wbp[4] = {-1, -1, -1, -1};
            if (!CANDS && tid < nacc) {
                const int per_r3 = G.nw[0] * G.nw[1] * G.nw[2];
                const unsigned long long key = s_key[tid];
                if (key == ~0ull) {
                    write_empty_track(a, i);
                } else {
                    const int c = (int)(key & (DV1 ? 0xfffffull : 127ull));
                    int slot = s_base[tid] + c / per_r3;
                    if (DV1) {
                        // the seed's item whose UTbX hit has the winning index
                        const int i3 = c / per_r3;
                        const int b1 = tid + 1 < nacc ? s_base[tid + 1] : n_items;
                        slot = s_base[tid];
                        for (int it = s_base[tid]; it < b1; ++it)
                            slot = (int)hidx_s[it_desc[it] & 0xffffu] == i3 ? it : slot;
                    }
                    int cw = c;
                    if (!DV1) {
                        const int base = s_base[tid];
                        const int nwin = (tid + 1 < nacc ? s_base[tid + 1] : n_items) - base;
                        if (nwin <= G.max_l3) {
                            const int p3w = (int)(it_desc[base + c / per_r3] & 0xffffu);
                            cw = first_window_rank(G, hu_s, hidx_s, s_c[tid], p3w) * per_r3 + c % per_r3;
                        }
                    }
                    const unsigned long long hp = it_hits[slot];
                    int bp[4];
#pragma unroll
                    for (int L = 0; L < 4; ++L) {
                        const int v = (int)((hp >> (16 * L)) & 0xffffull);
                        bp[L] = v == 0xffff ? -1 : v;
                    }
                    t = write_track(a, G, i, sd, s_c[tid], hu_s, hidx_s, bp, cw, nullptr);
                    won = true;
#pragma unroll
                    for (int L = 0; L < 4; ++L) wbp[L] = bp[L];
                }
            }
            if (!CANDS && a.fuse_mlp) {
                // the chunk's seed constants, keys and items are read: each
                // wavefront's feature tile goes there, and the network reads it
                lds_barrier();
                if (__ballot(won) != 0) {
                    float *T = reinterpret_cast<float *>(s_c) + (tid >> 6) * MLP_TILE;
                    float f[NF];
                    if (won) {
                        float hu4[4];
                        int mask = 0;
#pragma unroll
                        for (int L = 0; L < 4; ++L) {
                            hu4[L] = wbp[L] >= 0 ? hu_s[wbp[L]] : 0.0f;
                            mask |= wbp[L] >= 0 ? (1 << L) : 0;
                        }
                        ghost_features(G, t.x, t.y, t.tx, t.ty, t.qop, t.chi2, __popc(mask), sd.x, sd.y, sd.tx, sd.ty,
                                       sd.qop, hu4, mask, f);
                    }
                    mlp_tile_store(T, f, won);
                    float mw[MLP_LANE_WORDS];
                    mlp_lane_weights(a.W, mw);
                    const float sc_ = mlp_score_tile(mw, T, won);
                    if (won) {
                        t.score = sc_;
                        a.score[i] = sc_;
                    }
                }
            }
            const bool kept = VTX && won && t.score < a.score_max;
            if (VTX) {
                // kept tracks appended in slot order, split by seed charge
                int nk = s_nkept, nkp = s_nkpos;
                const int tcap = kernel_args<TrackKernArgs>().a.tcap;
                // (appending writes the list only: the row table is built by the vertexing)
                kept_append<BLOCK>(kept_carve(smem + kept_off, smem + kept_off, tcap), tcap, kept, sd.qop > 0.0f,
                                   make_float4(t.x, t.y, t.tx, t.ty), t.qop, i - s0,
                                   nk, nkp, s_wsum);
                lds_barrier();
                if (tid == 0) {
                    s_nkept = nk;
                    s_nkpos = nkp;
                }
            }
            lds_barrier();
            sc0 += nacc;
        }
        if (VTX) {
            const TrackKernArgs &Kv = kernel_args<TrackKernArgs>();
            vertex_event_block<BLOCK, XTR>(Kv.a, Kv.G, e, s0, s_nkept, s_nkpos,
                                           kept_carve(smem + kept_off, smem + Kv.a.krow_off, Kv.a.tcap), Kv.a.tcap,
                                           reinterpret_cast<int *>(s_c), s_wsum);
        }
    }
    const TrackArgs &a = kernel_args<TrackKernArgs>().a;
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

// ------------------------------------------------------------ event order
//
// Largest-first order of a batch for the persistent launch: uneven events
// are taken from the work counter biggest first, so that the launch does not
// end on one large event while the other workgroups idle.  A counting sort of
// a work estimate (seeds + hits / 8, in bins of two, the top bin open-ended),
// descending; events of one bin in any order (results do not depend on the
// processing order).  Workspace ws: [0, ORDER_BINS) bin counts,
// [ORDER_BINS, 2 ORDER_BINS) fill cursors, [2 ORDER_BINS] finished
// workgroups of k_order_place; all zero between calls (the last workgroup of
// k_order_place clears them).
constexpr int ORDER_BINS = 1024;
constexpr int ORDER_WS = 2 * ORDER_BINS + 64;   // ints ahead of the order array

__device__ __forceinline__ int order_bin(const int *seed_off, const int *hit_off, int e)
{
    const int s = seed_off[e + 1] - seed_off[e];
    const int h = hit_off[4 * e + 4] - hit_off[4 * e];
    const int cost = max(s, 0) + max(h, 0) / 8;
    return min(cost >> 1, ORDER_BINS - 1);
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_order_count(const int *seed_off, const int *hit_off, int n, int *ws)
{
    __shared__ int h[ORDER_BINS];
    for (int b = threadIdx.x; b < ORDER_BINS; b += BLOCK) h[b] = 0;
    __syncthreads();
    for (int e = blockIdx.x * BLOCK + threadIdx.x; e < n; e += gridDim.x * BLOCK)
        atomicAdd(&h[order_bin(seed_off, hit_off, e)], 1);
    __syncthreads();
    for (int b = threadIdx.x; b < ORDER_BINS; b += BLOCK)
        if (h[b]) atomicAdd(&ws[b], h[b]);
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_order_place(const int *seed_off, const int *hit_off, int n, int *ws,
                                                       int *order)
{
    static_assert(ORDER_BINS % BLOCK == 0, "whole bins per lane");
    constexpr int PER = ORDER_BINS / BLOCK;
    __shared__ int start[ORDER_BINS];
    __shared__ int s_wsum[BLOCK / 64];
    __shared__ int s_last;
    const int t = threadIdx.x;
    // lane t owns bins top - (t PER + j): a descending exclusive scan
    int v[PER], sum = 0;
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        v[j] = ws[ORDER_BINS - 1 - (t * PER + j)];
        sum += v[j];
    }
    int tot;
    int excl = block_exclusive_scan<BLOCK>(sum, s_wsum, &tot);
#pragma unroll
    for (int j = 0; j < PER; ++j) {
        start[ORDER_BINS - 1 - (t * PER + j)] = excl;
        excl += v[j];
    }
    __syncthreads();
    for (int e = blockIdx.x * BLOCK + t; e < n; e += gridDim.x * BLOCK) {
        const int b = order_bin(seed_off, hit_off, e);
        const int pos = start[b] + atomicAdd(&ws[ORDER_BINS + b], 1);
        if (pos < n) order[pos] = e;   // always, when the counts were zero on entry
    }
    __syncthreads();
    if (t == 0) {
        __threadfence();
        s_last = atomicAdd(&ws[2 * ORDER_BINS], 1) == (int)gridDim.x - 1;
    }
    __syncthreads();
    if (s_last) {
        __threadfence();
        for (int b = t; b < 2 * ORDER_BINS + 1; b += BLOCK) ws[b] = 0;
    }
}

// Sets n ints to v (graph-safe: a kernel, not a memset node).
__global__ void k_fill_i32(int *p, int v, int n)
{
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < n; k += gridDim.x * blockDim.x) p[k] = v;
}

// Marks every candidate row empty (nhits 0) before a candidate-scoring pass.
__global__ void k_clear_rows(int *r_nhits, long long n)
{
    for (long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (long long)gridDim.x * blockDim.x)
        r_nhits[k] = 0;
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
        // uniform trip count: the network runs on whole wavefronts
        for (int ib = s0; ib < s1; ib += BLOCK) {
            const int i = ib + (int)threadIdx.x;
            bool row = false;
            float f[NF];
            if (i < s1) {
                const int nh = a.nhits[i];
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
                if (nh > 0 && !hit_ok) atomicOr(a.flags, F_BAD_OFFSETS);
                row = nh > 0 && hit_ok;
                if (row)
                    ghost_features(G, a.x[i], a.y[i], a.tx[i], a.ty[i], a.qop[i], a.chi2[i], nh, a.sx[i], a.sy[i],
                                   a.stx[i], a.sty[i], a.sqop[i], hu4, has, f);
                else
                    a.score[i] = 0.0f;
            }
            if (__ballot(row) != 0) {
                float mw[MLP_LANE_WORDS];
                mlp_lane_weights(a.W, mw);
                const float sc = mlp_score_wave(mw, f, row);
                if (row) a.score[i] = sc;
            }
        }
    }
}

// ----------------------------------------------------------------- vertex

// Newton-Raphson point of closest approach in float64.  Offsets s, t are
// z - z_ref on each trajectory.  Returns false for (near-)parallel tracks or
// a singular Newton system.
__device__ __forceinline__ bool pca64(const DevGeom &G, double x1, double y1, double tx1, double ty1, double g1, double x2,
                             double y2, double tx2, double ty2, double g2, double &vx, double &vy, double &vz,
                             double &doca, double &s_out, double &t_out)
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
    s_out = s;
    t_out = t;
    return true;
}

// Invariant masses of a vertex (pi+ pi-, and p pi with the faster track as the
// proton; MeV) from the seed momenta and the trajectory tangents at the points
// of closest approach (offsets s, t from z_ref), then the four trigger-line
// networks (12 -> 32 ReLU -> 1 sigmoid, float32) on the pair and the vertex.
__device__ __forceinline__ void vertex_extras(const DevGeom &G, const float *WLg, float4 A, float4 B, double g1, double g2,
                                     float q1, float q2, double s, double t, float4 V, float out[6])
{
    const double MPI = 0.13957039, MPR = 0.93827209;
    const double d1x = (double)A.z + 2.0 * g1 * s, d1y = A.w, d2x = (double)B.z + 2.0 * g2 * t, d2y = B.w;
    const double n1 = sqrt(d1x * d1x + d1y * d1y + 1.0), n2 = sqrt(d2x * d2x + d2y * d2y + 1.0);
    const double p1 = 1.0 / fabs((double)q1), p2 = 1.0 / fabs((double)q2);
    const double Sx = p1 * d1x / n1 + p2 * d2x / n2;
    const double Sy = p1 * d1y / n1 + p2 * d2y / n2;
    const double Sz = p1 / n1 + p2 / n2;
    const double ss = Sx * Sx + Sy * Sy + Sz * Sz;
    const double e1 = sqrt(p1 * p1 + MPI * MPI), e2 = sqrt(p2 * p2 + MPI * MPI);
    double m2 = (e1 + e2) * (e1 + e2) - ss;
    const double mpipi = 1000.0 * sqrt(m2 > 0.0 ? m2 : 0.0);
    const double ep = p1 >= p2 ? sqrt(p1 * p1 + MPR * MPR) + e2 : sqrt(p2 * p2 + MPR * MPR) + e1;
    m2 = ep * ep - ss;
    const double mppi = 1000.0 * sqrt(m2 > 0.0 ? m2 : 0.0);
    out[0] = (float)mpipi;
    out[1] = (float)mppi;
    float f[LINE_NF];
    f[0] = (float)log(p1);
    f[1] = (float)log(p2);
    f[2] = (float)(d1x / 0.3);
    f[3] = (float)(d1y / 0.3);
    f[4] = (float)(d2x / 0.3);
    f[5] = (float)(d2y / 0.3);
    f[6] = V.z * 1e-3f;
    f[7] = sqrtf(V.x * V.x + V.y * V.y) * 0.01f;
    f[8] = V.w;
    f[9] = (float)((mpipi - 497.6) * 0.01);
    f[10] = (float)((mppi - 1115.7) * 0.01);
    f[11] = (float)sqrt(Sx * Sx + Sy * Sy);
    asm volatile("" : "+s"(WLg));
    cfloat *WL = (cfloat *)(WLg);
#pragma unroll
    for (int l = 0; l < 4; ++l) {
        cfloat *W = WL + l * LINE_NW, *b1 = W + LINE_NH * LINE_NF, *w2 = b1 + LINE_NH, *b2 = w2 + LINE_NH;
        float z = b2[0];
#pragma unroll
        for (int j = 0; j < LINE_NH; ++j) {
            float a = b1[j];
#pragma unroll
            for (int k = 0; k < LINE_NF; ++k) a = fmaf(W[j * LINE_NF + k], f[k], a);
            z = fmaf(w2[j], fmaxf(a, 0.0f), z);
        }
        out[2 + l] = 1.0f / (1.0f + __expf(-z));
    }
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Standalone vertexing (ds_vertex): a workgroup per event (work-stolen); the
// event's kept tracks (nhits > 0, score < score_max) are compacted into LDS in
// slot order, then the pairs go through vertex_event_block, the routine of the
// fused step.  LDS: kept tracks (kept_lds_bytes), their row table
// (kept_rows_bytes) and the survivor ring.
template <int BLOCK, bool XTR>
__global__ __launch_bounds__(BLOCK) void k_vertex(VertexArgs a, DevGeom G)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const Kept K = kept_carve(smem, smem + kept_lds_bytes(a.tcap), a.tcap);
    int *ring = reinterpret_cast<int *>(smem + kept_lds_bytes(a.tcap) + kept_rows_bytes(a.tcap));
    __shared__ int s_e;
    __shared__ int s_wsum[BLOCK / 64];
    const int tid = threadIdx.x;
    for (int iter = 0;; ++iter) {
        if (tid == 0) {
            if (a.ev_single >= 0)
                s_e = iter == 0 ? a.ev_single : a.n_events;
            else
                s_e = atomicAdd(&a.counter[0], 1);
        }
        lds_barrier();
        const int e = s_e;
        lds_barrier();   // s_e read by every wave before it is rewritten
        if (e >= a.n_events) break;
        const int s0 = a.seed_off[e], s1 = a.seed_off[e + 1];
        const bool ok = (0 <= s0) && (s0 <= s1) && (s1 <= a.n_seeds);
        if (!ok || s1 - s0 > a.tcap || s1 - s0 > a.max_seeds) {
            if (tid == 0) {
                atomicOr(a.flags, ok ? F_CAPACITY : F_BAD_OFFSETS);
                a.vcount[e] = 0;
            }
            continue;
        }
        // kept tracks, in slot order per seed charge
        int n = 0, np = 0;
        for (int base = s0; base < s1; base += BLOCK) {
            const int i = base + tid;
            const bool kept = (i < s1) && (a.nhits[i] > 0) && (a.score[i] < a.score_max);
            float4 v = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            float qv = 0.0f;
            bool positive = false;
            if (kept) {
                v = make_float4(a.x[i], a.y[i], a.tx[i], a.ty[i]);
                qv = a.qop[i];
                positive = a.sqop[i] > 0.0f;
            }
            kept_append<BLOCK>(K, a.tcap, kept, positive, v, qv, i - s0, n, np, s_wsum);
        }
        lds_barrier();   // the kept tracks are visible
        vertex_event_block<BLOCK, XTR>(a, G, e, s0, n, np, K, a.tcap, ring, s_wsum);
        lds_barrier();   // the event's LDS is free again
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

// Clone killing: one wavefront per event.  A found track is killed when
// another found track of the event shares more than two UT hits with it and
// has more hits, or as many and a lower chi2, or both equal and a lower slot.
// Decisions are taken on LDS copies, so the kills of one event do not depend
// on each other; a killed track is written as "no track".
template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_clone(CloneArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    unsigned char *wb = smem + (size_t)wid * (size_t)a.tcap * 16;
    unsigned long long *hp = reinterpret_cast<unsigned long long *>(wb);
    int *nh = reinterpret_cast<int *>(wb + (size_t)a.tcap * 8);
    float *c2 = reinterpret_cast<float *>(wb + (size_t)a.tcap * 12);
    const int waves = (int)gridDim.x * (BLOCK / 64);
    for (int e = (int)blockIdx.x * (BLOCK / 64) + wid; e < a.n_events; e += waves) {
        const int s0 = a.seed_off[e], s1 = a.seed_off[e + 1];
        const bool ok = (0 <= s0) && (s0 <= s1) && (s1 <= a.n_seeds);
        if (!ok || s1 - s0 > a.tcap || s1 - s0 > a.max_seeds) {
            if (lane == 0) atomicOr(a.flags, ok ? F_CAPACITY : F_BAD_OFFSETS);
            continue;
        }
        const int n = s1 - s0;
        for (int k = lane; k < n; k += 64) {
            const int i = s0 + k;
            const int h[4] = {a.h0[i], a.h1[i], a.h2[i], a.h3[i]};
            unsigned long long p = 0;
#pragma unroll
            for (int L = 0; L < 4; ++L)
                p |= (unsigned long long)(h[L] >= 0 ? ((unsigned)h[L] & 0xffffu) : 0xffffu) << (16 * L);
            hp[k] = p;
            nh[k] = a.nhits[i];
            c2[k] = a.chi2[i];
        }
        wave_sync();
        for (int k = lane; k < n; k += 64) {
            const int nk = nh[k];
            if (nk <= 0) continue;
            const unsigned long long pk = hp[k];
            const float ck = c2[k];
            bool killed = false;
            for (int j = 0; j < n && !killed; ++j) {
                const int nj = nh[j];
                if (j == k || nj <= 0) continue;
                const unsigned long long pj = hp[j];
                int shared = 0;
#pragma unroll
                for (int L = 0; L < 4; ++L) {
                    const unsigned hk = (unsigned)(pk >> (16 * L)) & 0xffffu;
                    shared += (hk != 0xffffu && hk == ((unsigned)(pj >> (16 * L)) & 0xffffu)) ? 1 : 0;
                }
                if (shared <= 2) continue;
                const float cj = c2[j];
                killed = nj > nk || (nj == nk && (cj < ck || (cj == ck && j < k)));
            }
            if (killed) {
                const int i = s0 + k;
                a.x[i] = 0.0f;
                a.y[i] = 0.0f;
                a.tx[i] = 0.0f;
                a.ty[i] = 0.0f;
                a.qop[i] = 0.0f;
                a.chi2[i] = 0.0f;
                if (a.score) a.score[i] = 0.0f;
                a.h0[i] = -1;
                a.h1[i] = -1;
                a.h2[i] = -1;
                a.h3[i] = -1;
                a.nhits[i] = 0;
                if (a.cand) a.cand[i] = -1;
            }
        }
        wave_sync();
    }
}

}  // namespace ds
