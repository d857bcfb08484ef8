/*
 * ds.h - C ABI of the MI355X (gfx950) Downstream tracking + two-track
 * vertexing library (Kholoimov et al., arXiv:2503.13092).
 *
 * The library implements the per-event hot path of the paper's Downstream
 * HLT1 algorithm ("The Downstream Algorithm", "Ghost-Killer Neural Network",
 * "Vertexing Two Downstream Tracks"): SciFi seeds are extrapolated through a
 * single magnet kink to the four UT layers, windows of x-sorted UT hits are
 * searched, candidates are scored with a least-squares chi2 and the best one
 * per seed is kept, a small MLP scores every track, and opposite-charge
 * pairs of kept tracks are vertexed by a Newton-Raphson point of closest
 * approach.
 *
 * Conventions for every call:
 *  - Units: mm, rad, GeV (q/p in GeV^-1).
 *  - Every array pointer inside ds_events / ds_tracks / ds_vertices is a
 *    DEVICE pointer owned by the caller.  The library never frees or keeps
 *    caller memory beyond the stream work it enqueues; buffers must stay
 *    valid until that work has completed.
 *  - Calls are asynchronous on `hip_stream` (a hipStream_t; NULL = the
 *    default stream).  A DS_OK return means the work was enqueued.
 *  - Host-detectable argument errors return DS_E_ARG before anything is
 *    enqueued.  Data errors found on the device (bad offsets, an event larger
 *    than the capacity the caller declared, non-finite inputs) are OR-ed into
 *    the caller's `flags` word (DS_F_* bits) and the affected event's outputs
 *    are written as "no track" / "no vertex"; read the word after a sync.
 *  - A HIP runtime failure returns DS_E_DEVICE; the context should then be
 *    destroyed and recreated.
 *  - Results are a pure function of the inputs and the loaded geometry: they
 *    do not depend on batch composition, launch mode or scheduling order.
 */
#ifndef DS_H
#define DS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ds_ctx ds_ctx;

typedef enum {
    DS_OK = 0,
    DS_E_ARG = 1,      /* invalid argument (null pointer, negative size, unsupported setting) */
    DS_E_STATE = 2,    /* geometry not loaded yet */
    DS_E_NOMEM = 3,    /* a library allocation failed */
    DS_E_CAPACITY = 4, /* a size exceeds what the library supports (LDS, streams, caps) */
    DS_E_DEVICE = 5    /* HIP runtime error */
} ds_status;

/* Launch modes of ds_find_tracks / ds_vertex / ds_process. */
enum {
    DS_MODE_PER_EVENT = 0,  /* plain path: one kernel launch per event per step */
    DS_MODE_PERSISTENT = 1, /* one persistent work-stealing launch per step */
    DS_MODE_GRAPH = 2       /* the persistent launch replayed from a cached hipGraph */
};

/* Device-written error bits (OR-ed into the caller's flags word). */
enum {
    DS_F_BAD_OFFSETS = 1, /* non-monotone or out-of-range seed/hit offsets: event skipped */
    DS_F_CAPACITY = 2,    /* event larger than max_*_per_event: event skipped */
    DS_F_NONFINITE = 4    /* non-finite hit (event skipped) or seed (seed gets no track) */
};

/*
 * Geometry and method settings (copied by ds_load_geometry).
 *  z_layer, tan_stereo : UTaX, UTaU, UTbV, UTbX planes and stereo tangents
 *                        (UT description, Fig. 2); hits measure
 *                        u = x - y*tan_stereo.
 *  z_magnet            : z of the single kink of the magnet-point model
 *                        (eq. 1 and the text after it).
 *  z_seed, z_ref       : z of the SciFi seed states; z of the output track
 *                        states (the UT midpoint z0 of eq. 4).
 *  kick, polarity      : the kink changes tx by polarity*kick*q/p.
 *  sigma_hit           : hit resolution of the chi2.
 *  w1_*, w2_*          : first (UTbX) and refined window half-widths,
 *                        W = c0 + c1*|q/p| ("Algorithm Design": windows are
 *                        functions of momentum).
 *  u_min, u_max        : range of u used to bin hits for the window lookup
 *                        (hits outside still work; they land in edge bins).
 *  max_l3, n_closest   : up to max_l3 (<= 16) closest UTbX hits, and the
 *                        n_closest[L] (<= 2) closest hits in UTaX, UTaU, UTbV.
 *  gamma_*, fringe_polarity : eq. 3, gamma = -fringe_polarity*(c0 + c1*q/p[MeV^-1]);
 *                        fringe_polarity = 0 gives straight trajectories.
 *  newton_iters        : Newton-Raphson steps of the vertex fit (0..16).
 *  doca_max            : a vertex is kept if its DOCA < doca_max.
 *  ghost_threshold     : a track is kept if its ghost score < threshold
 *                        ("Ghost Rejection"); used by ds_process.
 *  clone_kill          : nonzero: ds_process kills clones (ds_kill_clones)
 *                        between track finding and the ghost-killer.
 *  algorithm           : 0 = Dv0 (momentum window in UTbX, up to max_l3
 *                        closest hits); 1 = Dv1, the improved version of
 *                        "Algorithm Design": no momentum window, every UTbX
 *                        hit of a compatible Y sector is joined to the magnet
 *                        point and the line must meet a UTaX hit (the axial
 *                        triplet); stereo hits, fit and selection as in Dv0.
 *                        Dv1 needs ds_events.hit_sector.  Candidate rows
 *                        (ds_score_candidates) always follow Dv0.
 *  n_sectors, sector_y0,
 *  sector_h, sector_tol: Dv1 Y sectors: sector k of a layer is the band
 *                        [sector_y0 + k*sector_h, sector_y0 + (k+1)*sector_h),
 *                        k < n_sectors (<= 15).  A seed reaches the sectors
 *                        that overlap [y - sector_tol, y + sector_tol], y its
 *                        straight-line height at the layer;
 *                        2*sector_tol < sector_h.  Ignored when algorithm = 0.
 *                        Dv1 candidate index: ((i3*nw0 + i0)*nw1 + i1)*nw2 + i2
 *                        with i3 the UTbX hit's index in its layer run.
 */
typedef struct {
    double z_layer[4];
    double tan_stereo[4];
    double z_magnet, z_seed, z_ref;
    double kick, polarity;
    double sigma_hit;
    double w1_c0, w1_c1, w2_c0, w2_c1;
    double u_min, u_max;
    int32_t max_l3;
    int32_t n_closest[3];
    double gamma_c0, gamma_c1, fringe_polarity;
    int32_t newton_iters;
    double doca_max;
    double ghost_threshold;
    int32_t clone_kill;
    int32_t algorithm;
    int32_t n_sectors;
    double sector_y0, sector_h, sector_tol;
} ds_geometry;

/*
 * A batch of events (structure of arrays, event-major).
 *  seed_off [n_events+1]     : seeds of event e are [seed_off[e], seed_off[e+1]).
 *  sx..sqop [n_seeds]        : SciFi seed state (x, y, tx, ty, q/p) at z_seed.
 *  hit_off  [4*n_events+1]   : hits of event e, layer L are
 *                              [hit_off[4e+L], hit_off[4e+L+1]).
 *  hu       [n_hits]         : hit coordinate u, any order within a run.
 *  n_seeds, n_hits           : array lengths; every offset must lie in [0, len].
 *  max_seeds_per_event,
 *  max_hits_per_event        : caller's upper bounds (all four layers for hits);
 *                              they size on-chip buffers.  An event above a
 *                              bound is flagged DS_F_CAPACITY and skipped.
 *  hit_sector [n_hits]       : Y sector of each hit (Dv1; nullable for Dv0).
 *                              A sector id >= n_sectors is never compatible.
 */
typedef struct {
    int32_t n_events;
    int32_t n_seeds;
    int32_t n_hits;
    int32_t max_seeds_per_event;
    int32_t max_hits_per_event;
    const int32_t *seed_off;
    const float *sx, *sy, *stx, *sty, *sqop;
    const int32_t *hit_off;
    const float *hu;
    const uint8_t *hit_sector;
} ds_events;

/*
 * Tracks: one slot per seed [n_seeds] (state at z_ref).
 *  hit[L]  : index of the chosen hit within its (event, layer) run, -1 = none.
 *  nhits   : 0 = no track for this seed (all other fields then 0 / -1).
 *  cand    : index of the selected candidate (nullable), -1 if none.
 *  score   : ghost-killer response, written by ds_ghost_kill or by
 *            ds_find_tracks with fuse_mlp != 0 (0 for seeds without a track).
 *  flags   : [1] device word, OR-ed (never cleared by the library).
 */
typedef struct {
    float *x, *y, *tx, *ty, *qop, *chi2, *score;
    int32_t *hit[4];
    int32_t *nhits;
    int32_t *cand;
    int32_t *flags;
} ds_tracks;

/*
 * Vertices: at most cap_per_event per event, (i, j)-ordered, i < j being
 * seed slots within the event.  count[n_events]; i, j, x, y, z, doca
 * [n_events*cap_per_event].  overflow [1]: number of vertices dropped beyond
 * the cap, added to (never cleared by the library).  flags [1]: OR-ed.
 * m_pipi, m_ppi, line[4] (all or none; nullable; need ds_load_lines): the
 * pair's invariant mass in MeV under the pi+ pi- and p pi (faster track =
 * proton) hypotheses, from the seed momenta and the trajectory tangents at
 * the points of closest approach (mass after the vertex correction, Fig. 18),
 * and the four trigger-line network responses ("Expected Physics Impact").
 */
typedef struct {
    int32_t cap_per_event;
    int32_t *count;
    int32_t *i, *j;
    float *x, *y, *z, *doca;
    int32_t *overflow;
    int32_t *flags;
    float *m_pipi, *m_ppi;
    float *line[4];
} ds_vertices;

/*
 * Every enumerated candidate, scored: the ghost-killer is trained on all
 * candidates found with wide windows and clone killing off ("Ghost-Killer
 * Neural Network").  Row r = seed * ds_candidate_slots() + candidate index
 * holds that candidate as if it were the selected track (float32 state at
 * z_ref, chi2, hits, ghost score); rows of candidates that do not exist or
 * are invalid have nhits = 0.  capacity >= n_seeds * ds_candidate_slots().
 */
typedef struct {
    int32_t capacity;
    int32_t *seed, *cand, *nhits;
    int32_t *hit[4];
    float *x, *y, *tx, *ty, *qop, *chi2, *score;
    int32_t *flags;
} ds_candidates;

/* Create a context on HIP device `device`.  *ctx is set on DS_OK. */
ds_status ds_create(ds_ctx **ctx, int device);

/* Destroy a context (waits for nothing; the caller syncs its streams first). */
void ds_destroy(ds_ctx *ctx);

/*
 * Load the geometry and the ghost-killer parameters.  `mlp_weights` is a
 * HOST array of n_weights = 1121 floats: W1[32][17], b1[32], W2[16][32],
 * b2[16], W3[1][16], b3[1] (row-major; the network of "Ghost-Killer Neural
 * Network" widened to 17 -> 32 -> 16 -> 1, ReLU hidden layers, sigmoid
 * output).  Copied to device memory, which stays resident.  Synchronous:
 * first waits for all work on the context's device (launches already
 * enqueued keep the old geometry and weights), then replaces both.
 */
ds_status ds_load_geometry(ds_ctx *ctx, const ds_geometry *g, const float *mlp_weights, size_t n_weights);

/*
 * Load the four trigger-line networks ("Expected Physics Impact": one hidden
 * layer of 32 nodes, one output): a HOST array of 4 x 449 floats, each
 * W1[32][12], b1[32], W2[1][32], b2[1] row-major; ReLU hidden, sigmoid out.
 * Inputs per vertex: ln p1, ln p2 (GeV), the two tracks' tangent slopes
 * (dx/dz, dy/dz)/0.3 at the vertex, z/1000, transverse radius/100, DOCA,
 * (m_pipi - 497.6)/100, (m_ppi - 1115.7)/100, pair pT (GeV).  Synchronous.
 */
ds_status ds_load_lines(ds_ctx *ctx, const float *line_weights, size_t n_weights);

/*
 * Track finding ("The Downstream Algorithm", Dv0, or Dv1's triplet search when
 * the loaded geometry says algorithm = 1): one track slot per seed.
 * mode = DS_MODE_*; fuse_mlp != 0 also writes the ghost-killer score.
 * DS_E_ARG if Dv1 is loaded and ev->hit_sector is null.
 */
ds_status ds_find_tracks(ds_ctx *ctx, const ds_events *ev, const ds_tracks *out, int mode, int fuse_mlp,
                         void *hip_stream);

/*
 * Clone killing ("Algorithm Design": among track pairs sharing more than two
 * UT hits the lower-scored candidate is killed).  Within each event, a found
 * track is killed when another found track shares more than two hits with it
 * (same hit in the same layer) and is better: more hits, else lower chi2,
 * else lower seed slot.  All pairs are judged on the tracks as found; a
 * killed track is rewritten as "no track" (nhits 0, hits -1, state 0, score 0).
 * Uses trk->flags for device-side offset/capacity errors.
 */
ds_status ds_kill_clones(ds_ctx *ctx, const ds_events *ev, const ds_tracks *trk, void *hip_stream);

/* Candidate rows per seed for the loaded geometry: max_l3 * prod(max(n_closest, 1)); 0 before loading. */
int ds_candidate_slots(ds_ctx *ctx);

/* Score every valid candidate of every seed (see ds_candidates). */
ds_status ds_score_candidates(ds_ctx *ctx, const ds_events *ev, const ds_candidates *out, void *hip_stream);

/* Ghost-killer scores of the tracks in `trk` ("Ghost-Killer Neural Network":
 * a small fully connected network scores each reconstructed track; "Ghost
 * Rejection": tracks scoring at or above the threshold are dropped
 * downstream).  Reads the stored track, the seed and the chosen hits; writes
 * trk->score (0 for seeds without a track).  Device-side offset errors and
 * hit indices outside their run set DS_F_BAD_OFFSETS in trk->flags. */
ds_status ds_ghost_kill(ds_ctx *ctx, const ds_events *ev, const ds_tracks *trk, void *hip_stream);

/*
 * Two-track vertexing ("Vertexing Two Downstream Tracks"): pairs of tracks
 * with nhits > 0 and score < score_max and opposite seed charge; Newton-
 * Raphson PCA of the eq. 4 trajectories; kept if DOCA < doca_max.
 */
ds_status ds_vertex(ds_ctx *ctx, const ds_events *ev, const ds_tracks *trk, float score_max,
                    const ds_vertices *out, int mode, void *hip_stream);

/* The whole step: ds_find_tracks (fused MLP) then ds_vertex with
 * score_max = ghost_threshold (or `score_max` if it is not NaN), as one fused
 * launch or as the two (ds_set_step_fusion); with geometry clone_kill set:
 * ds_find_tracks, ds_kill_clones, ds_ghost_kill, ds_vertex.  In
 * DS_MODE_GRAPH all launches are one cached hipGraph. */
ds_status ds_process(ds_ctx *ctx, const ds_events *ev, const ds_tracks *trk, float score_max,
                     const ds_vertices *out, int mode, void *hip_stream);

/*
 * ds_process without allocation, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same step as ds_process in DS_MODE_PERSISTENT, with
 * the same results, the event order set by ds_set_event_order, and no
 * hipMalloc / hipFree or other allocation in the call.  Its work counters
 * and largest-first order live in a static device array of the library
 * (1.06 MB per device, held until the process ends), cleared at the start of
 * each call by a fill kernel on hip_stream.  Every call on one device shares
 * that array: calls that overlap on one device (on any streams or contexts)
 * race and must not be issued.  The caller passes inputs and outputs as for
 * ds_process.  DS_E_CAPACITY when n_events > DS_STATIC_MAX_EVENTS.
 */
#define DS_STATIC_MAX_EVENTS 262144
ds_status ds_process_static(ds_ctx *ctx, const ds_events *ev, const ds_tracks *trk, float score_max,
                            const ds_vertices *out, void *hip_stream);

/*
 * Launch tuning (used by the autotuner).  kernel: 0 = tracking, 1 = vertexing.
 * block: threads per workgroup (64, 128, 192 (tracking only), 256, 512); wg_per_cu: persistent
 * workgroups per compute unit (1..16); bins: hit bins per layer for the
 * window lookup (tracking only; 64..4096, power of two).  0 keeps a value.
 */
ds_status ds_set_launch(ds_ctx *ctx, int kernel, int block, int wg_per_cu, int bins);

/* Current launch settings of `kernel` (same meaning as ds_set_launch). */
ds_status ds_get_launch(ds_ctx *ctx, int kernel, int *block, int *wg_per_cu, int *bins);

/* Event order of the persistent tracking launch. */
enum {
    DS_ORDER_INPUT = 0,        /* events taken from the work counter in batch order */
    DS_ORDER_LARGEST_FIRST = 1 /* largest first (seeds + hits/8), so that uneven batches do not end on
                                  one large event ("GPU Implementation": events of a slice differ in size) */
};

/*
 * Set / read the event order of ds_find_tracks and ds_process in
 * DS_MODE_PERSISTENT and DS_MODE_GRAPH (per-event launches ignore it).
 * Largest-first adds two small launches that sort the batch's events by a
 * work estimate into a per-stream workspace the library allocates (and grows,
 * after draining the device, when a larger batch comes).  Results do not
 * depend on the order; only speed does.
 */
ds_status ds_set_event_order(ds_ctx *ctx, int order);
ds_status ds_get_event_order(ds_ctx *ctx, int *order);

/*
 * Set / read how ds_process and ds_process_static run the step (without
 * clone killing) in DS_MODE_PERSISTENT and DS_MODE_GRAPH: fused = 1 (the
 * default) runs tracking, ghost-killer and vertexing in one launch, the kept
 * tracks of an event never leaving LDS; fused = 0 runs ds_find_tracks (with
 * the ghost-killer fused) and then ds_vertex, whose kernel holds fewer
 * registers and more events per compute unit, which pays where pairs
 * dominate.  Results are identical; only speed differs.
 */
ds_status ds_set_step_fusion(ds_ctx *ctx, int fused);
ds_status ds_get_step_fusion(ds_ctx *ctx, int *fused);

/* Human-readable name of a status code (static string). */
const char *ds_status_str(ds_status s);

#ifdef __cplusplus
}
#endif

#endif /* DS_H */
