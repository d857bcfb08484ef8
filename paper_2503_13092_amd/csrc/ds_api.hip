// Host side of the Downstream tracking + vertexing library: the C ABI of
// include/ds.h, argument validation, launch configuration and the three
// launch modes (one launch per event, one persistent work-stealing launch,
// or that launch replayed from a cached hipGraph).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "ds.h"
#include "ds_kernels.h"

namespace {

constexpr int MAX_STREAM_SLOTS = 64;
constexpr int MAX_GRAPHS = 64;
constexpr int ITEMS_PER_SEED = 3;
constexpr int CLONE_BLOCK = 256;
constexpr size_t LDS_LIMIT = 160 * 1024 - 256;   // gfx950: 160 KiB per workgroup, minus static use
constexpr float PRESCREEN_MARGIN = 0.1f;         // mm, see the float32 error bound of the pair prescreen

struct Launch {
    int block, wg_per_cu, bins;
};

constexpr int MAX_DEVICES = 64;
constexpr int STATIC_HDR = 64;   // ints: [0, 2) tracking and [2, 4) vertexing work counters
constexpr int STATIC_INTS = STATIC_HDR + ds::ORDER_WS + DS_STATIC_MAX_EVENTS;

// Largest-first event order of one stream slot: ORDER_WS ints of bin counts
// and cursors (zero between calls), then the order of up to `cap` events.
struct OrderWs {
    int *p = nullptr;
    int cap = 0;
};

struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;   // recorded after every replay: the graph is idle once it has completed
    uint64_t last_use = 0;
};

// Destroy a cached graph once its last replay has finished (a replay may
// still be running on a caller stream).
void release_graph(GraphEntry &g)
{
    if (g.done) {
        (void)hipEventSynchronize(g.done);
        (void)hipEventDestroy(g.done);
    }
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    g = GraphEntry{};
}

}  // namespace

// ds_process_static's workspace, for callers that cannot allocate: the work
// counters, then the largest-first order's bins and cursors (ORDER_WS ints),
// then the order of up to DS_STATIC_MAX_EVENTS events; 1.06 MB.  Every device
// the library runs on holds its own copy until the process ends.  On the host
// the name stands for no device address: host code uses only the address
// static_scratch() looked up for the device.
static __device__ __align__(256) int scratch[STATIC_INTS];

namespace {

std::mutex g_scratch_mu;
int *g_scratch[MAX_DEVICES] = {};

// The current device's copy of `scratch` (looked up once per device; the
// device must be current).
ds_status static_scratch(int device, int **p)
{
    if (device < 0 || device >= MAX_DEVICES) return DS_E_CAPACITY;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[device]) {
        void *q = nullptr;
        if (hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)) != hipSuccess || !q) return DS_E_DEVICE;
        g_scratch[device] = static_cast<int *>(q);
    }
    *p = g_scratch[device];
    return DS_OK;
}

}  // namespace

struct ds_ctx {
    int device = 0;
    int *scratch = nullptr;    // this device's static workspace (ds_process_static)
    int n_cu = 256;
    bool loaded = false;
    ds::DevGeom G{};
    double u_min = -1000.0, u_max = 1000.0;
    double ghost_threshold = 0.5;
    bool clone_kill = false;
    int algorithm = 0;             // 0: Dv0 window search, 1: Dv1 triplet search
    float *d_W = nullptr;    // ghost-killer weights, per-lane MFMA order (mlp_lane_layout)
    float *d_Wrow = nullptr; // the same, row-major (the candidate rows' per-lane network)
    float *d_WL = nullptr;   // trigger-line networks
    int *d_counters = nullptr;  // [MAX_STREAM_SLOTS][4]
    std::map<void *, int> slots;
    OrderWs order_ws[MAX_STREAM_SLOTS];
    int event_order = DS_ORDER_INPUT;   // persistent launches: DS_ORDER_*
    int fused_step = 1;                 // ds_process: one fused launch (1) or tracking then vertexing (0)
    Launch trk{256, 3, 1024};  // three resident workgroups per CU (168 VGPRs, ~50 KB LDS): one grid wave
    Launch vtx{256, 4, 0};    // workgroup per event, four resident per CU
    hipStream_t capture = nullptr;
    std::map<std::string, GraphEntry> graphs;
    uint64_t tick = 0;
    std::mutex mu;
};

namespace {

ds_status dev_err(hipError_t e) { return e == hipSuccess ? DS_OK : DS_E_DEVICE; }

size_t round16(size_t v) { return (v + 15) & ~size_t(15); }

// Dynamic LDS of the tracking kernel, mirroring its carve: hits, bucket
// bounds, then the seed constants ... item buffers (one region: phase C's
// feature tiles and the fused vertexing's survivor ring and row table reuse
// it), then the fused vertexing's kept tracks.
struct TrackLayout {
    size_t sc;      // seed constants: start of the reusable region
    size_t kept;    // its end: the kept tracks
    size_t total;
};

TrackLayout track_layout(int hcap, int nb, int nb3, int block, int icap, int tcap)
{
    TrackLayout L;
    size_t off = (size_t)hcap * 4;
    off = round16(off + (size_t)hcap * 2);
    off = round16(off + (size_t)(3 * nb + nb3 + 1) * 2);
    L.sc = off;
    off += (size_t)block * sizeof(ds::SeedConst);
    off += (size_t)block * 8;
    off = round16(off + (size_t)block * 4);
    off = round16(off + (size_t)icap * 4);
    L.kept = round16(off + (size_t)icap * 8);
    L.total = L.kept + ds::kept_lds_bytes(tcap);
    return L;
}

// k_vertex: the event's kept tracks, their row table, then the survivor ring of the pair loop
size_t vertex_lds(int tcap, int block)
{
    return ds::kept_lds_bytes(tcap) + ds::kept_rows_bytes(tcap) + sizeof(int) * (size_t)ds::vtx_ring_ints(block);
}

int round_up(int v, int m) { return ((v + m - 1) / m) * m; }

ds_status slot_for(ds_ctx *c, void *stream, int **counters, int *slot = nullptr)
{
    auto it = c->slots.find(stream);
    int s;
    if (it == c->slots.end()) {
        if ((int)c->slots.size() >= MAX_STREAM_SLOTS) return DS_E_CAPACITY;
        s = (int)c->slots.size();
        c->slots[stream] = s;
    } else {
        s = it->second;
    }
    *counters = c->d_counters + 4 * s;
    if (slot) *slot = s;
    return DS_OK;
}

// The largest-first workspace of a stream slot for n events (grown on demand:
// launches in flight may hold the old buffer, so the device is drained first,
// and cached graphs that name it are dropped).
ds_status order_workspace(ds_ctx *c, int slot, int n, int **ws)
{
    OrderWs &o = c->order_ws[slot];
    if (o.cap < n) {
        if (o.p) {
            if (hipDeviceSynchronize() != hipSuccess) return DS_E_DEVICE;
            for (auto &g : c->graphs) release_graph(g.second);
            c->graphs.clear();
            (void)hipFree(o.p);
            o = OrderWs{};
        }
        const int cap = std::max(n, 1024);
        int *p = nullptr;
        if (hipMalloc(&p, sizeof(int) * ((size_t)ds::ORDER_WS + (size_t)cap)) != hipSuccess) return DS_E_NOMEM;
        if (hipMemset(p, 0, sizeof(int) * (size_t)ds::ORDER_WS) != hipSuccess) {
            (void)hipFree(p);
            return DS_E_DEVICE;
        }
        o.p = p;
        o.cap = cap;
    }
    *ws = o.p;
    return DS_OK;
}

ds_status check_events(const ds_events *ev)
{
    if (!ev) return DS_E_ARG;
    if (ev->n_events < 0 || ev->n_seeds < 0 || ev->n_hits < 0 || ev->max_seeds_per_event < 0 ||
        ev->max_hits_per_event < 0)
        return DS_E_ARG;
    if (ev->n_events == 0) return DS_OK;
    if (!ev->seed_off || !ev->hit_off) return DS_E_ARG;
    if (ev->n_seeds > 0 && (!ev->sx || !ev->sy || !ev->stx || !ev->sty || !ev->sqop)) return DS_E_ARG;
    if (ev->n_hits > 0 && !ev->hu) return DS_E_ARG;
    return DS_OK;
}

ds_status check_extras(const ds_ctx *c, const ds_vertices *v)
{
    const bool any = v->m_pipi || v->m_ppi || v->line[0] || v->line[1] || v->line[2] || v->line[3];
    if (!any) return DS_OK;
    if (!(v->m_pipi && v->m_ppi && v->line[0] && v->line[1] && v->line[2] && v->line[3])) return DS_E_ARG;
    return c->d_WL ? DS_OK : DS_E_STATE;
}

ds_status check_tracks(const ds_tracks *t, int n_seeds, bool need_score)
{
    if (!t || !t->flags) return DS_E_ARG;
    if (n_seeds == 0) return DS_OK;
    if (!t->x || !t->y || !t->tx || !t->ty || !t->qop || !t->chi2 || !t->nhits) return DS_E_ARG;
    for (int L = 0; L < 4; ++L)
        if (!t->hit[L]) return DS_E_ARG;
    if (need_score && !t->score) return DS_E_ARG;
    return DS_OK;
}

template <typename K>
void append_bytes(std::string &key, const K &v)
{
    key.append(reinterpret_cast<const char *>(&v), sizeof(K));
}

// ---------------------------------------------------------------- kernels

template <int B>
hipError_t launch_track_b(const ds::TrackArgs &a, const ds::DevGeom &G, int grid, size_t lds, hipStream_t s)
{
    const ds::TrackKernArgs k{a, G};
    if (a.cmax > 0)
        hipLaunchKernelGGL((ds::k_track<B, true, false, false>), dim3(grid), dim3(B), lds, s, k);
    else if (a.hsec && a.vcount && a.m_pipi)
        hipLaunchKernelGGL((ds::k_track<B, false, true, true, true>), dim3(grid), dim3(B), lds, s, k);
    else if (a.hsec && a.vcount)
        hipLaunchKernelGGL((ds::k_track<B, false, true, true>), dim3(grid), dim3(B), lds, s, k);
    else if (a.hsec)
        hipLaunchKernelGGL((ds::k_track<B, false, false, true>), dim3(grid), dim3(B), lds, s, k);
    else if (a.vcount && a.m_pipi)
        hipLaunchKernelGGL((ds::k_track<B, false, true, false, true>), dim3(grid), dim3(B), lds, s, k);
    else if (a.vcount)
        hipLaunchKernelGGL((ds::k_track<B, false, true, false>), dim3(grid), dim3(B), lds, s, k);
    else
        hipLaunchKernelGGL((ds::k_track<B, false, false, false>), dim3(grid), dim3(B), lds, s, k);
    return hipGetLastError();
}

hipError_t launch_track(int block, const ds::TrackArgs &a, const ds::DevGeom &G, int grid, size_t lds,
                        hipStream_t s)
{
    switch (block) {
    case 64: return launch_track_b<64>(a, G, grid, lds, s);
    case 128: return launch_track_b<128>(a, G, grid, lds, s);
    case 192: return launch_track_b<192>(a, G, grid, lds, s);
    case 256: return launch_track_b<256>(a, G, grid, lds, s);
    default: return launch_track_b<512>(a, G, grid, lds, s);
    }
}

template <int B>
hipError_t launch_vertex_b(const ds::VertexArgs &a, const ds::DevGeom &G, int grid, size_t lds, hipStream_t s)
{
    if (a.m_pipi)
        hipLaunchKernelGGL((ds::k_vertex<B, true>), dim3(grid), dim3(B), lds, s, a, G);
    else
        hipLaunchKernelGGL((ds::k_vertex<B, false>), dim3(grid), dim3(B), lds, s, a, G);
    return hipGetLastError();
}

hipError_t launch_vertex(int block, const ds::VertexArgs &a, const ds::DevGeom &G, int grid, size_t lds,
                         hipStream_t s)
{
    switch (block) {
    case 64: return launch_vertex_b<64>(a, G, grid, lds, s);
    case 128: return launch_vertex_b<128>(a, G, grid, lds, s);
    case 256: return launch_vertex_b<256>(a, G, grid, lds, s);
    default: return launch_vertex_b<512>(a, G, grid, lds, s);
    }
}

// Allow every instantiation the full LDS of a gfx950 workgroup.
hipError_t set_kernel_attributes()
{
    const void *fns[] = {
#define DS_TRACK_FNS(B)                                                                                     \
    reinterpret_cast<const void *>(&ds::k_track<B, false, false, false>),                                   \
        reinterpret_cast<const void *>(&ds::k_track<B, true, false, false>),                                \
        reinterpret_cast<const void *>(&ds::k_track<B, false, true, false>),                                \
        reinterpret_cast<const void *>(&ds::k_track<B, false, false, true>),                                \
        reinterpret_cast<const void *>(&ds::k_track<B, false, true, true>),                                 \
        reinterpret_cast<const void *>(&ds::k_track<B, false, true, false, true>),                          \
        reinterpret_cast<const void *>(&ds::k_track<B, false, true, true, true>)
        DS_TRACK_FNS(64), DS_TRACK_FNS(128), DS_TRACK_FNS(192), DS_TRACK_FNS(256), DS_TRACK_FNS(512),
#undef DS_TRACK_FNS
        reinterpret_cast<const void *>(&ds::k_vertex<64, false>),
        reinterpret_cast<const void *>(&ds::k_vertex<128, false>),
        reinterpret_cast<const void *>(&ds::k_vertex<256, false>),
        reinterpret_cast<const void *>(&ds::k_vertex<512, false>),
        reinterpret_cast<const void *>(&ds::k_vertex<64, true>),
        reinterpret_cast<const void *>(&ds::k_vertex<128, true>),
        reinterpret_cast<const void *>(&ds::k_vertex<256, true>),
        reinterpret_cast<const void *>(&ds::k_vertex<512, true>),
        reinterpret_cast<const void *>(&ds::k_clone<CLONE_BLOCK>)};
    for (const void *f : fns) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)LDS_LIMIT);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// A prepared launch: arguments, shape, and the per-event variant.
struct TrackPlan {
    ds::TrackArgs a;
    int block, grid;
    size_t lds;
    int *order_ws = nullptr;   // persistent launch in largest-first order: its workspace
    int n_cu = 256;
};

struct VertexPlan {
    ds::VertexArgs a;
    int block, grid;
    size_t lds;
};

ds_status plan_track(ds_ctx *c, const ds_events *ev, const ds_tracks *out, int fuse, int *counters, TrackPlan *p,
                     bool vertex_fused = false, bool cand_rows = false)
{
    // Dv1 buckets hits by (layer, Y sector, u bin) plus one bucket per layer
    // for sector ids out of range; candidate rows always follow Dv0
    const bool dv1 = c->algorithm == 1 && !cand_rows;
    if (dv1 && !ev->hit_sector) return DS_E_ARG;
    // Dv1 reads layer 3 by whole sectors (one u bin each); layers 0-2 share the
    // rest of the 4 x bins bucket budget
    const int nsec = c->G.nsec;
    const int nbu = dv1 ? std::max(4, (4 * c->trk.bins - nsec - 4) / (3 * nsec)) : c->trk.bins;
    const int nb = dv1 ? nsec * nbu + 1 : nbu;
    const int nbu3 = dv1 ? 1 : nbu, nb3 = dv1 ? nsec + 1 : nb;
    int hcap = round_up(std::max(ev->max_hits_per_event, 1), 16);
    if (hcap > 65535) return DS_E_CAPACITY;   // 16-bit LDS positions and bucket bounds
    const int block = c->trk.block;
    // items per chunk: room for ITEMS_PER_SEED per seed; a chunk shrinks when its seeds need more
    const int icap = std::max(block * ITEMS_PER_SEED, ds::MAX_L3);
    const int tcap = vertex_fused ? round_up(std::max(ev->max_seeds_per_event, 1), 16) : 0;
    if (tcap > 32767) return DS_E_CAPACITY;   // 15-bit kept-track indices
    const TrackLayout L = track_layout(hcap, nb, nb3, block, icap, tcap);
    size_t lds = L.total;
    // the network's feature tiles reuse the seed-constant ... item region
    const size_t region = L.kept - L.sc;
    if (region < (size_t)(block / 64) * ds::MLP_TILE * 4) return DS_E_CAPACITY;
    // ... and so do the fused pair loop's survivor ring and, where it fits
    // after the ring, the kept tracks' row table (else it gets its own space)
    int krow_off = 0;
    if (vertex_fused) {
        const size_t ring = round16(sizeof(int) * (size_t)ds::vtx_ring_ints(block));
        if (region < ring) return DS_E_CAPACITY;
        if (region - ring >= ds::kept_rows_bytes(tcap)) {
            krow_off = (int)(L.sc + ring);
        } else {
            krow_off = (int)lds;
            lds += ds::kept_rows_bytes(tcap);
        }
    }
    if (lds > LDS_LIMIT) return DS_E_CAPACITY;
    ds::TrackArgs &a = p->a;
    std::memset(&a, 0, sizeof(a));
    a.n_events = ev->n_events;
    a.n_seeds = ev->n_seeds;
    a.n_hits = ev->n_hits;
    a.max_seeds = ev->max_seeds_per_event;
    a.max_hits = ev->max_hits_per_event;
    a.seed_off = ev->seed_off;
    a.sx = ev->sx;
    a.sy = ev->sy;
    a.stx = ev->stx;
    a.sty = ev->sty;
    a.sqop = ev->sqop;
    a.hit_off = ev->hit_off;
    a.hu = ev->hu;
    a.x = out->x;
    a.y = out->y;
    a.tx = out->tx;
    a.ty = out->ty;
    a.qop = out->qop;
    a.chi2 = out->chi2;
    a.score = out->score;
    a.h0 = out->hit[0];
    a.h1 = out->hit[1];
    a.h2 = out->hit[2];
    a.h3 = out->hit[3];
    a.nhits = out->nhits;
    a.cand = out->cand;
    a.flags = out->flags;
    a.counter = counters;
    a.W = c->d_W;
    a.fuse_mlp = fuse ? 1 : 0;
    a.ev_single = -1;
    a.hcap = hcap;
    a.icap = icap;
    a.tcap = tcap;
    a.krow_off = krow_off;
    a.nb = nb;
    a.nbu = nbu;
    a.u0 = (float)c->u_min;
    a.inv_bw = (float)((double)nbu / (c->u_max - c->u_min));
    a.nb3 = nb3;
    a.nbu3 = nbu3;
    a.inv_bw3 = (float)((double)nbu3 / (c->u_max - c->u_min));
    a.hsec = dv1 ? ev->hit_sector : nullptr;
    p->block = block;
    p->grid = std::max(1, std::min(ev->n_events, c->n_cu * c->trk.wg_per_cu));
    p->lds = lds;
    p->n_cu = c->n_cu;
    p->order_ws = nullptr;
    return DS_OK;
}

// A persistent launch takes the events largest first when the context says so
// (ws: the slot's workspace; the order kernels run ahead of the launch).
void set_order(TrackPlan &p, int *ws)
{
    p.order_ws = ws;
    p.a.order = ws ? ws + ds::ORDER_WS : nullptr;
}

ds_status plan_order(ds_ctx *c, int slot, int mode, TrackPlan &p)
{
    if (mode == DS_MODE_PER_EVENT || c->event_order != DS_ORDER_LARGEST_FIRST || p.a.n_events < 2) return DS_OK;
    int *ws = nullptr;
    const ds_status st = order_workspace(c, slot, p.a.n_events, &ws);
    if (st == DS_OK) set_order(p, ws);
    return st;
}

ds_status plan_vertex(ds_ctx *c, const ds_events *ev, const ds_tracks *trk, float score_max, const ds_vertices *out,
                      int *counters, VertexPlan *p)
{
    int tcap = round_up(std::max(ev->max_seeds_per_event, 1), 64);
    if (tcap > 32767) return DS_E_CAPACITY;   // 15-bit kept-track indices
    size_t lds = vertex_lds(tcap, c->vtx.block);
    if (lds > LDS_LIMIT) return DS_E_CAPACITY;
    ds::VertexArgs &a = p->a;
    std::memset(&a, 0, sizeof(a));
    a.n_events = ev->n_events;
    a.n_seeds = ev->n_seeds;
    a.max_seeds = ev->max_seeds_per_event;
    a.seed_off = ev->seed_off;
    a.sqop = ev->sqop;
    a.x = trk->x;
    a.y = trk->y;
    a.tx = trk->tx;
    a.ty = trk->ty;
    a.qop = trk->qop;
    a.score = trk->score;
    a.nhits = trk->nhits;
    a.score_max = score_max;
    a.vcap = out->cap_per_event;
    a.vcount = out->count;
    a.vi = out->i;
    a.vj = out->j;
    a.vx = out->x;
    a.vy = out->y;
    a.vz = out->z;
    a.vdoca = out->doca;
    a.voverflow = out->overflow;
    a.flags = out->flags;
    a.counter = counters + 2;
    a.ev_single = -1;
    a.tcap = tcap;
    a.m_pipi = out->m_pipi;
    a.m_ppi = out->m_ppi;
    a.line0 = out->line[0];
    a.line1 = out->line[1];
    a.line2 = out->line[2];
    a.line3 = out->line[3];
    a.WL = c->d_WL;
    p->block = c->vtx.block;
    p->grid = std::max(1, std::min(ev->n_events, c->n_cu * c->vtx.wg_per_cu));
    p->lds = lds;
    return DS_OK;
}

ds::GhostArgs ghost_args(ds_ctx *c, const ds_events *ev, const ds_tracks *trk)
{
    ds::GhostArgs a;
    std::memset(&a, 0, sizeof(a));
    a.n_events = ev->n_events;
    a.n_seeds = ev->n_seeds;
    a.n_hits = ev->n_hits;
    a.seed_off = ev->seed_off;
    a.sx = ev->sx;
    a.sy = ev->sy;
    a.stx = ev->stx;
    a.sty = ev->sty;
    a.sqop = ev->sqop;
    a.hit_off = ev->hit_off;
    a.hu = ev->hu;
    a.x = trk->x;
    a.y = trk->y;
    a.tx = trk->tx;
    a.ty = trk->ty;
    a.qop = trk->qop;
    a.chi2 = trk->chi2;
    a.h0 = trk->hit[0];
    a.h1 = trk->hit[1];
    a.h2 = trk->hit[2];
    a.h3 = trk->hit[3];
    a.nhits = trk->nhits;
    a.score = trk->score;
    a.flags = trk->flags;
    a.W = c->d_W;
    return a;
}

hipError_t launch_ghost(ds_ctx *c, const ds::GhostArgs &a, hipStream_t s)
{
    const int grid = std::max(1, std::min(a.n_events, c->n_cu * 8));
    hipLaunchKernelGGL(ds::k_ghost<128>, dim3(grid), dim3(128), 0, s, a, c->G);
    return hipGetLastError();
}

ds_status clone_args(const ds_events *ev, const ds_tracks *trk, ds::CloneArgs *a, size_t *lds)
{
    std::memset(a, 0, sizeof(*a));
    const int tcap = round_up(std::max(ev->max_seeds_per_event, 1), 64);
    *lds = (size_t)tcap * 16 * (CLONE_BLOCK / 64);
    if (*lds > LDS_LIMIT) return DS_E_CAPACITY;
    a->n_events = ev->n_events;
    a->n_seeds = ev->n_seeds;
    a->max_seeds = ev->max_seeds_per_event;
    a->seed_off = ev->seed_off;
    a->x = trk->x;
    a->y = trk->y;
    a->tx = trk->tx;
    a->ty = trk->ty;
    a->qop = trk->qop;
    a->chi2 = trk->chi2;
    a->score = trk->score;
    a->h0 = trk->hit[0];
    a->h1 = trk->hit[1];
    a->h2 = trk->hit[2];
    a->h3 = trk->hit[3];
    a->nhits = trk->nhits;
    a->cand = trk->cand;
    a->flags = trk->flags;
    a->tcap = tcap;
    return DS_OK;
}

hipError_t launch_clone(ds_ctx *c, const ds::CloneArgs &a, size_t lds, hipStream_t s)
{
    const int waves = CLONE_BLOCK / 64;
    const int grid = std::max(1, std::min((a.n_events + waves - 1) / waves, c->n_cu * 8));
    hipLaunchKernelGGL(ds::k_clone<CLONE_BLOCK>, dim3(grid), dim3(CLONE_BLOCK), lds, s, a);
    return hipGetLastError();
}

// The largest-first order of the batch into ws + ORDER_WS (two small launches).
hipError_t launch_order(const ds::TrackArgs &a, int *ws, int n_cu, hipStream_t s)
{
    constexpr int B = 256;
    const int grid = std::max(1, std::min((a.n_events + B - 1) / B, 4 * n_cu));
    hipLaunchKernelGGL(ds::k_order_count<B>, dim3(grid), dim3(B), 0, s, a.seed_off, a.hit_off, a.n_events, ws);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(ds::k_order_place<B>, dim3(grid), dim3(B), 0, s, a.seed_off, a.hit_off, a.n_events, ws,
                       ws + ds::ORDER_WS);
    return hipGetLastError();
}

hipError_t run_track(ds_ctx *c, const TrackPlan &p, int mode, hipStream_t s)
{
    if (mode == DS_MODE_PER_EVENT) {
        ds::TrackArgs a = p.a;
        for (int e = 0; e < a.n_events; ++e) {
            a.ev_single = e;
            hipError_t err = launch_track(p.block, a, c->G, 1, p.lds, s);
            if (err != hipSuccess) return err;
        }
        return hipSuccess;
    }
    if (p.a.order) {
        hipError_t e = launch_order(p.a, p.order_ws, p.n_cu, s);
        if (e != hipSuccess) return e;
    }
    return launch_track(p.block, p.a, c->G, p.grid, p.lds, s);
}

hipError_t run_vertex(ds_ctx *c, const VertexPlan &p, int mode, hipStream_t s)
{
    if (mode == DS_MODE_PER_EVENT) {
        ds::VertexArgs a = p.a;
        for (int e = 0; e < a.n_events; ++e) {
            a.ev_single = e;
            hipError_t err = launch_vertex(p.block, a, c->G, 1, p.lds, s);
            if (err != hipSuccess) return err;
        }
        return hipSuccess;
    }
    return launch_vertex(p.block, p.a, c->G, p.grid, p.lds, s);
}

// Run `body` (which enqueues persistent launches on the given stream) either
// directly or through a hipGraph cached under `key`.
template <typename F>
ds_status run_maybe_graph(ds_ctx *c, int mode, const std::string &key, hipStream_t s, F body)
{
    if (mode != DS_MODE_GRAPH) return dev_err(body(s));
    auto it = c->graphs.find(key);
    if (it == c->graphs.end()) {
        if ((int)c->graphs.size() >= MAX_GRAPHS) {
            auto victim = c->graphs.begin();
            for (auto g = c->graphs.begin(); g != c->graphs.end(); ++g)
                if (g->second.last_use < victim->second.last_use) victim = g;
            release_graph(victim->second);
            c->graphs.erase(victim);
        }
        GraphEntry ge;
        hipError_t err = hipStreamBeginCapture(c->capture, hipStreamCaptureModeRelaxed);
        if (err != hipSuccess) return DS_E_DEVICE;
        hipError_t berr = body(c->capture);
        err = hipStreamEndCapture(c->capture, &ge.graph);
        if (berr != hipSuccess || err != hipSuccess) {
            if (ge.graph) (void)hipGraphDestroy(ge.graph);
            return DS_E_DEVICE;
        }
        err = hipGraphInstantiate(&ge.exec, ge.graph, nullptr, nullptr, 0);
        if (err == hipSuccess) err = hipEventCreateWithFlags(&ge.done, hipEventDisableTiming);
        if (err != hipSuccess) {
            release_graph(ge);
            return DS_E_DEVICE;
        }
        it = c->graphs.emplace(key, ge).first;
    }
    it->second.last_use = ++c->tick;
    hipError_t err = hipGraphLaunch(it->second.exec, s);
    if (err == hipSuccess) err = hipEventRecord(it->second.done, s);
    return dev_err(err);
}

std::string graph_key(int kind, const void *args, size_t n, int block, int grid, size_t lds)
{
    std::string key;
    append_bytes(key, kind);
    key.append(reinterpret_cast<const char *>(args), n);
    append_bytes(key, block);
    append_bytes(key, grid);
    append_bytes(key, lds);
    return key;
}

// Argument checks of ds_process / ds_process_static (host side, before any launch).
ds_status check_process(ds_ctx *c, const ds_events *ev, const ds_tracks *trk, const ds_vertices *out, int mode)
{
    if (!c) return DS_E_ARG;
    if (!c->loaded) return DS_E_STATE;
    if (mode < DS_MODE_PER_EVENT || mode > DS_MODE_GRAPH) return DS_E_ARG;
    ds_status st = check_events(ev);
    if (st != DS_OK) return st;
    st = check_tracks(trk, ev->n_seeds, true);
    if (st != DS_OK) return st;
    if (!out || out->cap_per_event < 0 || !out->overflow || !out->flags) return DS_E_ARG;
    if (ev->n_events == 0) return DS_OK;
    if (!out->count) return DS_E_ARG;
    if (out->cap_per_event > 0 && (!out->i || !out->j || !out->x || !out->y || !out->z || !out->doca))
        return DS_E_ARG;
    return check_extras(c, out);
}

// Enqueue the whole step on s: work counters at `counters` ([0, 2) tracking,
// [2, 4) vertexing), the largest-first order in order_ws (null: input order).
// Outside DS_MODE_GRAPH nothing here allocates (no graph keys are built).
ds_status process_enqueue(ds_ctx *c, const ds_events *ev, const ds_tracks *trk, float score_max,
                          const ds_vertices *out, int mode, hipStream_t s, int *counters, int *order_ws)
{
    const bool ck = c->clone_kill;
    TrackPlan tp;
    ds_status st = plan_track(c, ev, trk, ck ? 0 : 1, counters, &tp);
    if (st != DS_OK) return st;
    if (mode != DS_MODE_PER_EVENT) set_order(tp, order_ws);
    VertexPlan vp;
    st = plan_vertex(c, ev, trk, score_max, out, counters, &vp);
    if (st != DS_OK) return st;
    ds::CloneArgs ca;
    size_t clds = 0;
    ds::GhostArgs ga = ghost_args(c, ev, trk);
    if (ck) {
        st = clone_args(ev, trk, &ca, &clds);
        if (st != DS_OK) return st;
    }
    if (!ck && mode != DS_MODE_PER_EVENT && c->fused_step) {
        // one launch: tracking, ghost-killer and vertexing fused per event
        TrackPlan fp;
        st = plan_track(c, ev, trk, 1, counters, &fp, true);
        if (st != DS_OK) return st;
        set_order(fp, tp.order_ws);
        ds::TrackArgs &a = fp.a;
        a.score_max = score_max;
        a.vcap = out->cap_per_event;
        a.vcount = out->count;
        a.vi = out->i;
        a.vj = out->j;
        a.vx = out->x;
        a.vy = out->y;
        a.vz = out->z;
        a.vdoca = out->doca;
        a.voverflow = out->overflow;
        a.vflags = out->flags;
        a.m_pipi = out->m_pipi;
        a.m_ppi = out->m_ppi;
        a.line0 = out->line[0];
        a.line1 = out->line[1];
        a.line2 = out->line[2];
        a.line3 = out->line[3];
        a.WL = c->d_WL;
        auto body = [&](hipStream_t ss) { return run_track(c, fp, mode, ss); };
        if (mode != DS_MODE_GRAPH) return dev_err(body(s));
        return run_maybe_graph(c, mode, graph_key(5, &a, sizeof(a), fp.block, fp.grid, fp.lds), s, body);
    }
    auto body = [&](hipStream_t ss) {
        hipError_t e = run_track(c, tp, mode, ss);
        if (e != hipSuccess) return e;
        if (ck) {
            e = launch_clone(c, ca, clds, ss);
            if (e != hipSuccess) return e;
            e = launch_ghost(c, ga, ss);
            if (e != hipSuccess) return e;
        }
        return run_vertex(c, vp, mode, ss);
    };
    if (mode != DS_MODE_GRAPH) return dev_err(body(s));
    std::string key = graph_key(ck ? 4 : 2, &tp.a, sizeof(tp.a), tp.block, tp.grid, tp.lds);
    key += graph_key(3, &vp.a, sizeof(vp.a), vp.block, vp.grid, vp.lds);
    return run_maybe_graph(c, mode, key, s, body);
}

}  // namespace

extern "C" {

const char *ds_status_str(ds_status s)
{
    switch (s) {
    case DS_OK: return "DS_OK";
    case DS_E_ARG: return "DS_E_ARG: invalid argument";
    case DS_E_STATE: return "DS_E_STATE: geometry not loaded";
    case DS_E_NOMEM: return "DS_E_NOMEM: allocation failed";
    case DS_E_CAPACITY: return "DS_E_CAPACITY: size beyond library capacity";
    case DS_E_DEVICE: return "DS_E_DEVICE: HIP runtime error";
    }
    return "unknown ds_status";
}

ds_status ds_create(ds_ctx **ctx, int device)
{
    if (!ctx) return DS_E_ARG;
    *ctx = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return DS_E_ARG;
    if (hipSetDevice(device) != hipSuccess) return DS_E_DEVICE;
    ds_ctx *c = new (std::nothrow) ds_ctx();
    if (!c) return DS_E_NOMEM;
    c->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        c->n_cu = prop.multiProcessorCount;
    ds_status sst = static_scratch(device, &c->scratch);
    if (sst != DS_OK) {
        delete c;
        return sst;
    }
    if (hipMalloc(&c->d_counters, sizeof(int) * 4 * MAX_STREAM_SLOTS) != hipSuccess) {
        delete c;
        return DS_E_NOMEM;
    }
    if (set_kernel_attributes() != hipSuccess ||
        hipMemset(c->d_counters, 0, sizeof(int) * 4 * MAX_STREAM_SLOTS) != hipSuccess ||
        hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking) != hipSuccess) {
        (void)hipFree(c->d_counters);
        delete c;
        return DS_E_DEVICE;
    }
    *ctx = c;
    return DS_OK;
}

void ds_destroy(ds_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    for (auto &g : c->graphs) release_graph(g.second);
    if (c->d_W) (void)hipFree(c->d_W);
    if (c->d_Wrow) (void)hipFree(c->d_Wrow);
    if (c->d_WL) (void)hipFree(c->d_WL);
    if (c->d_counters) (void)hipFree(c->d_counters);
    for (auto &o : c->order_ws)
        if (o.p) (void)hipFree(o.p);
    if (c->capture) (void)hipStreamDestroy(c->capture);
    delete c;
}

ds_status ds_load_geometry(ds_ctx *c, const ds_geometry *g, const float *w, size_t nw)
{
    if (!c || !g || !w || nw != (size_t)ds::NWEIGHTS) return DS_E_ARG;
    if (g->max_l3 < 0 || g->max_l3 > ds::MAX_L3 || g->newton_iters < 0 || g->newton_iters > 16) return DS_E_ARG;
    for (int L = 0; L < 3; ++L)
        if (g->n_closest[L] < 0 || g->n_closest[L] > ds::MAX_CLOSEST) return DS_E_ARG;
    if (!(g->u_max > g->u_min) || !(g->sigma_hit > 0.0) || g->z_magnet == g->z_layer[3]) return DS_E_ARG;
    for (int L = 0; L < 3; ++L)
        if (!(g->z_layer[L] < g->z_layer[L + 1])) return DS_E_ARG;
    if (g->algorithm != 0 && g->algorithm != 1) return DS_E_ARG;
    // Dv1: at most 15 sectors (4-bit spans) and a tolerance band narrower than
    // a sector, so that a seed is compatible with at most two of them
    if (g->algorithm == 1 && (g->n_sectors < 1 || g->n_sectors > 15 || !(g->sector_h > 0.0) ||
                              !(g->sector_tol >= 0.0) || !(2.0 * g->sector_tol < g->sector_h) ||
                              !std::isfinite(g->sector_y0)))
        return DS_E_ARG;
    std::lock_guard<std::mutex> lock(c->mu);
    if (hipSetDevice(c->device) != hipSuccess) return DS_E_DEVICE;
    // launches already enqueued on any stream read the resident weights and
    // the cached graphs: let them finish before either is replaced
    if (hipDeviceSynchronize() != hipSuccess) return DS_E_DEVICE;
    ds::DevGeom G{};
    for (int L = 0; L < 4; ++L) {
        G.zl[L] = g->z_layer[L];
        G.tana[L] = g->tan_stereo[L];
        G.dz[L] = g->z_layer[L] - g->z_ref;
    }
    G.zm = g->z_magnet;
    G.zs = g->z_seed;
    G.zref = g->z_ref;
    G.mk = g->polarity * g->kick;
    G.inv_sigma2 = 1.0 / (g->sigma_hit * g->sigma_hit);
    G.inv_5sigma = 1.0 / (5.0 * g->sigma_hit);
    G.w1c0 = g->w1_c0;
    G.w1c1 = g->w1_c1;
    G.w2c0 = g->w2_c0;
    G.w2c1 = g->w2_c1;
    for (int L = 0; L < 3; ++L) G.ffac[L] = (g->z_magnet - g->z_layer[L]) / (g->z_magnet - g->z_layer[3]);
    const int masks[4] = {11, 13, 14, 15};
    for (int k = 0; k < 4; ++k) {
        double n = 0, sz = 0, szz = 0;
        for (int L = 0; L < 4; ++L)
            if ((masks[k] >> L) & 1) {
                n += 1;
                sz += G.dz[L];
                szz += G.dz[L] * G.dz[L];
            }
        G.fit_sz[k] = sz;
        G.fit_inv_det[k] = 1.0 / (n * szz - sz * sz);
        G.fit_inv_n[k] = 1.0 / n;
    }
    G.zm_ref = g->z_magnet - g->z_ref;
    G.zm_seed = g->z_magnet - g->z_seed;
    G.zref_seed = g->z_ref - g->z_seed;
    G.gc0 = g->gamma_c0;
    G.gc1 = g->gamma_c1;
    G.fp = g->fringe_polarity;
    G.doca_max = g->doca_max;
    const float thr = (float)g->doca_max + PRESCREEN_MARGIN;
    G.prescreen_thr2 = thr * thr;
    G.max_l3 = g->max_l3;
    for (int L = 0; L < 3; ++L) {
        G.ncl[L] = g->n_closest[L];
        G.nw[L] = std::max(g->n_closest[L], 1);
    }
    G.newton_iters = g->newton_iters;
    G.nsec = g->algorithm == 1 ? g->n_sectors : 1;
    G.sec_y0 = g->sector_y0;
    G.sec_h = g->algorithm == 1 ? g->sector_h : 1.0;
    G.sec_tol = g->sector_tol;
    // the ghost-killer network is evaluated on the matrix cores: its weights go
    // to the device in the per-lane order of the MFMA operands
    std::vector<float> wm(ds::MLP_WM);
    ds::mlp_lane_layout(w, wm.data());
    if (!c->d_W && hipMalloc(&c->d_W, sizeof(float) * ds::MLP_WM) != hipSuccess) return DS_E_NOMEM;
    if (hipMemcpy(c->d_W, wm.data(), sizeof(float) * ds::MLP_WM, hipMemcpyHostToDevice) != hipSuccess)
        return DS_E_DEVICE;
    if (!c->d_Wrow && hipMalloc(&c->d_Wrow, sizeof(float) * ds::NWEIGHTS) != hipSuccess) return DS_E_NOMEM;
    if (hipMemcpy(c->d_Wrow, w, sizeof(float) * ds::NWEIGHTS, hipMemcpyHostToDevice) != hipSuccess)
        return DS_E_DEVICE;
    c->G = G;
    c->u_min = g->u_min;
    c->u_max = g->u_max;
    c->ghost_threshold = g->ghost_threshold;
    c->clone_kill = g->clone_kill != 0;
    c->algorithm = g->algorithm;
    // cached graphs hold the old geometry as kernel arguments
    for (auto &e : c->graphs) release_graph(e.second);
    c->graphs.clear();
    c->loaded = true;
    return DS_OK;
}

ds_status ds_find_tracks(ds_ctx *c, const ds_events *ev, const ds_tracks *out, int mode, int fuse, void *stream)
{
    if (!c) return DS_E_ARG;
    if (!c->loaded) return DS_E_STATE;
    if (mode < DS_MODE_PER_EVENT || mode > DS_MODE_GRAPH) return DS_E_ARG;
    ds_status st = check_events(ev);
    if (st != DS_OK) return st;
    st = check_tracks(out, ev->n_seeds, fuse != 0);
    if (st != DS_OK) return st;
    if (ev->n_events == 0) return DS_OK;
    std::lock_guard<std::mutex> lock(c->mu);
    if (hipSetDevice(c->device) != hipSuccess) return DS_E_DEVICE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int *counters, slot;
    st = slot_for(c, stream, &counters, &slot);
    if (st != DS_OK) return st;
    TrackPlan p;
    st = plan_track(c, ev, out, fuse, counters, &p);
    if (st != DS_OK) return st;
    st = plan_order(c, slot, mode, p);
    if (st != DS_OK) return st;
    std::string key = graph_key(0, &p.a, sizeof(p.a), p.block, p.grid, p.lds);
    return run_maybe_graph(c, mode, key, s, [&](hipStream_t ss) { return run_track(c, p, mode, ss); });
}

ds_status ds_ghost_kill(ds_ctx *c, const ds_events *ev, const ds_tracks *trk, void *stream)
{
    if (!c) return DS_E_ARG;
    if (!c->loaded) return DS_E_STATE;
    ds_status st = check_events(ev);
    if (st != DS_OK) return st;
    st = check_tracks(trk, ev->n_seeds, true);
    if (st != DS_OK) return st;
    if (ev->n_events == 0) return DS_OK;
    std::lock_guard<std::mutex> lock(c->mu);
    if (hipSetDevice(c->device) != hipSuccess) return DS_E_DEVICE;
    return dev_err(launch_ghost(c, ghost_args(c, ev, trk), reinterpret_cast<hipStream_t>(stream)));
}

ds_status ds_kill_clones(ds_ctx *c, const ds_events *ev, const ds_tracks *trk, void *stream)
{
    if (!c) return DS_E_ARG;
    if (!c->loaded) return DS_E_STATE;
    ds_status st = check_events(ev);
    if (st != DS_OK) return st;
    st = check_tracks(trk, ev->n_seeds, false);
    if (st != DS_OK) return st;
    if (ev->n_events == 0) return DS_OK;
    std::lock_guard<std::mutex> lock(c->mu);
    if (hipSetDevice(c->device) != hipSuccess) return DS_E_DEVICE;
    ds::CloneArgs a;
    size_t lds;
    st = clone_args(ev, trk, &a, &lds);
    if (st != DS_OK) return st;
    return dev_err(launch_clone(c, a, lds, reinterpret_cast<hipStream_t>(stream)));
}

int ds_candidate_slots(ds_ctx *c)
{
    if (!c || !c->loaded) return 0;
    return c->G.max_l3 * c->G.nw[0] * c->G.nw[1] * c->G.nw[2];
}

ds_status ds_score_candidates(ds_ctx *c, const ds_events *ev, const ds_candidates *out, void *stream)
{
    if (!c) return DS_E_ARG;
    if (!c->loaded) return DS_E_STATE;
    ds_status st = check_events(ev);
    if (st != DS_OK) return st;
    if (!out || !out->flags || out->capacity < 0) return DS_E_ARG;
    if (ev->n_events == 0) return DS_OK;
    const int cmax = c->G.max_l3 * c->G.nw[0] * c->G.nw[1] * c->G.nw[2];
    if (cmax <= 0) return DS_OK;
    if ((long long)out->capacity < (long long)ev->n_seeds * cmax) return DS_E_CAPACITY;
    if (ev->n_seeds > 0) {
        if (!out->seed || !out->cand || !out->nhits || !out->x || !out->y || !out->tx || !out->ty || !out->qop ||
            !out->chi2 || !out->score)
            return DS_E_ARG;
        for (int L = 0; L < 4; ++L)
            if (!out->hit[L]) return DS_E_ARG;
    }
    std::lock_guard<std::mutex> lock(c->mu);
    if (hipSetDevice(c->device) != hipSuccess) return DS_E_DEVICE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int *counters;
    st = slot_for(c, stream, &counters);
    if (st != DS_OK) return st;
    ds_tracks none;
    std::memset(&none, 0, sizeof(none));
    none.flags = out->flags;
    TrackPlan p;
    st = plan_track(c, ev, &none, 0, counters, &p, false, true);
    if (st != DS_OK) return st;
    p.a.cmax = cmax;
    p.a.r_seed = out->seed;
    p.a.r_cand = out->cand;
    p.a.r_nhits = out->nhits;
    p.a.r_h0 = out->hit[0];
    p.a.r_h1 = out->hit[1];
    p.a.r_h2 = out->hit[2];
    p.a.r_h3 = out->hit[3];
    p.a.r_x = out->x;
    p.a.r_y = out->y;
    p.a.r_tx = out->tx;
    p.a.r_ty = out->ty;
    p.a.r_qop = out->qop;
    p.a.r_chi2 = out->chi2;
    p.a.r_score = out->score;
    p.a.Wrow = c->d_Wrow;   // each candidate is scored where it is written
    const long long rows = (long long)ev->n_seeds * cmax;
    if (rows > 0) {
        const int grid = (int)std::min<long long>((rows + 255) / 256, (long long)c->n_cu * 16);
        hipLaunchKernelGGL(ds::k_clear_rows, dim3(grid), dim3(256), 0, s, out->nhits, rows);
        if (hipGetLastError() != hipSuccess) return DS_E_DEVICE;
    }
    return dev_err(run_track(c, p, DS_MODE_PERSISTENT, s));
}

ds_status ds_vertex(ds_ctx *c, const ds_events *ev, const ds_tracks *trk, float score_max, const ds_vertices *out,
                    int mode, void *stream)
{
    if (!c) return DS_E_ARG;
    if (!c->loaded) return DS_E_STATE;
    if (mode < DS_MODE_PER_EVENT || mode > DS_MODE_GRAPH) return DS_E_ARG;
    ds_status st = check_events(ev);
    if (st != DS_OK) return st;
    st = check_tracks(trk, ev->n_seeds, true);
    if (st != DS_OK) return st;
    if (!out || out->cap_per_event < 0 || !out->overflow || !out->flags) return DS_E_ARG;
    if (ev->n_events == 0) return DS_OK;
    if (!out->count) return DS_E_ARG;
    if (out->cap_per_event > 0 && (!out->i || !out->j || !out->x || !out->y || !out->z || !out->doca))
        return DS_E_ARG;
    st = check_extras(c, out);
    if (st != DS_OK) return st;
    std::lock_guard<std::mutex> lock(c->mu);
    if (hipSetDevice(c->device) != hipSuccess) return DS_E_DEVICE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int *counters;
    st = slot_for(c, stream, &counters);
    if (st != DS_OK) return st;
    VertexPlan p;
    st = plan_vertex(c, ev, trk, score_max, out, counters, &p);
    if (st != DS_OK) return st;
    std::string key = graph_key(1, &p.a, sizeof(p.a), p.block, p.grid, p.lds);
    return run_maybe_graph(c, mode, key, s, [&](hipStream_t ss) { return run_vertex(c, p, mode, ss); });
}

ds_status ds_process(ds_ctx *c, const ds_events *ev, const ds_tracks *trk, float score_max, const ds_vertices *out,
                     int mode, void *stream)
{
    ds_status st = check_process(c, ev, trk, out, mode);
    if (st != DS_OK || ev->n_events == 0) return st;
    if (std::isnan(score_max)) score_max = (float)c->ghost_threshold;
    std::lock_guard<std::mutex> lock(c->mu);
    if (hipSetDevice(c->device) != hipSuccess) return DS_E_DEVICE;
    int *counters, slot;
    st = slot_for(c, stream, &counters, &slot);
    if (st != DS_OK) return st;
    int *order_ws = nullptr;
    if (mode != DS_MODE_PER_EVENT && c->event_order == DS_ORDER_LARGEST_FIRST && ev->n_events >= 2) {
        st = order_workspace(c, slot, ev->n_events, &order_ws);
        if (st != DS_OK) return st;
    }
    return process_enqueue(c, ev, trk, score_max, out, mode, reinterpret_cast<hipStream_t>(stream), counters,
                           order_ws);
}

ds_status ds_process_static(ds_ctx *c, const ds_events *ev, const ds_tracks *trk, float score_max,
                            const ds_vertices *out, void *stream)
{
    ds_status st = check_process(c, ev, trk, out, DS_MODE_PERSISTENT);
    if (st != DS_OK) return st;
    if (ev->n_events > DS_STATIC_MAX_EVENTS) return DS_E_CAPACITY;
    if (ev->n_events == 0) return DS_OK;
    if (std::isnan(score_max)) score_max = (float)c->ghost_threshold;
    std::lock_guard<std::mutex> lock(c->mu);
    if (hipSetDevice(c->device) != hipSuccess) return DS_E_DEVICE;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // the device's static array (its address, looked up at ds_create): work
    // counters and order bins start at zero (a fill kernel, not a memset node,
    // so that a caller may capture the call)
    int *sp = c->scratch;
    hipLaunchKernelGGL(ds::k_fill_i32, dim3(8), dim3(256), 0, s, sp, 0, STATIC_HDR + ds::ORDER_WS);
    if (hipGetLastError() != hipSuccess) return DS_E_DEVICE;
    int *order_ws = (c->event_order == DS_ORDER_LARGEST_FIRST && ev->n_events >= 2) ? sp + STATIC_HDR : nullptr;
    return process_enqueue(c, ev, trk, score_max, out, DS_MODE_PERSISTENT, s, sp, order_ws);
}

ds_status ds_load_lines(ds_ctx *c, const float *w, size_t nw)
{
    if (!c || !w || nw != (size_t)(4 * ds::LINE_NW)) return DS_E_ARG;
    std::lock_guard<std::mutex> lock(c->mu);
    if (hipSetDevice(c->device) != hipSuccess) return DS_E_DEVICE;
    if (!c->d_WL && hipMalloc(&c->d_WL, sizeof(float) * 4 * ds::LINE_NW) != hipSuccess) return DS_E_NOMEM;
    if (hipMemcpy(c->d_WL, w, sizeof(float) * 4 * ds::LINE_NW, hipMemcpyHostToDevice) != hipSuccess)
        return DS_E_DEVICE;
    return DS_OK;
}

ds_status ds_set_launch(ds_ctx *c, int kernel, int block, int wg_per_cu, int bins)
{
    if (!c || (kernel != 0 && kernel != 1)) return DS_E_ARG;
    if (block != 0 && block != 64 && block != 128 && block != 192 && block != 256 && block != 512) return DS_E_ARG;
    if (kernel == 1 && block == 192) return DS_E_ARG;   // tracking only
    if (wg_per_cu < 0 || wg_per_cu > 16) return DS_E_ARG;
    if (bins != 0 && (kernel != 0 || bins < 64 || bins > 4096 || (bins & (bins - 1)))) return DS_E_ARG;
    std::lock_guard<std::mutex> lock(c->mu);
    Launch &L = kernel == 0 ? c->trk : c->vtx;
    Launch n = L;
    if (block) n.block = block;
    if (wg_per_cu) n.wg_per_cu = wg_per_cu;
    if (bins) n.bins = bins;
    L = n;
    return DS_OK;
}

ds_status ds_set_event_order(ds_ctx *c, int order)
{
    if (!c || (order != DS_ORDER_INPUT && order != DS_ORDER_LARGEST_FIRST)) return DS_E_ARG;
    std::lock_guard<std::mutex> lock(c->mu);
    c->event_order = order;
    return DS_OK;
}

ds_status ds_set_step_fusion(ds_ctx *c, int fused)
{
    if (!c || (fused != 0 && fused != 1)) return DS_E_ARG;
    std::lock_guard<std::mutex> lock(c->mu);
    c->fused_step = fused;
    return DS_OK;
}

ds_status ds_get_step_fusion(ds_ctx *c, int *fused)
{
    if (!c || !fused) return DS_E_ARG;
    std::lock_guard<std::mutex> lock(c->mu);
    *fused = c->fused_step;
    return DS_OK;
}

ds_status ds_get_event_order(ds_ctx *c, int *order)
{
    if (!c || !order) return DS_E_ARG;
    std::lock_guard<std::mutex> lock(c->mu);
    *order = c->event_order;
    return DS_OK;
}

ds_status ds_get_launch(ds_ctx *c, int kernel, int *block, int *wg_per_cu, int *bins)
{
    if (!c || (kernel != 0 && kernel != 1) || !block || !wg_per_cu || !bins) return DS_E_ARG;
    std::lock_guard<std::mutex> lock(c->mu);
    const Launch &L = kernel == 0 ? c->trk : c->vtx;
    *block = L.block;
    *wg_per_cu = L.wg_per_cu;
    *bins = L.bins;
    return DS_OK;
}

}  // extern "C"
