// C ABI of batched stepping: many independent instances advanced by one
// persistent launch captured in a HIP graph, or by one launch per iteration
// that covers every instance (declared in include/teuk.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cstdio>
#include <cstdlib>
#include <fstream>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/teuk.h"
#include "ctx.h"
#include "kernels.h"

#ifndef TEUK_SOURCE_HASH
#define TEUK_SOURCE_HASH "unversioned"
#endif

using teuk_detail::fail;
using teuk_detail::hip_fail;
using teuk_detail::kSourceBatch;

namespace {

constexpr int kGraphCache = 8;          // captured (rounds, seg_rows) graphs kept per batch
constexpr double kWaitLimitSeconds = 2.0;

struct BatchGraph {
    int64_t rounds = 0;
    int seg = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

}  // namespace

struct teuk_batch {
    std::vector<teuk_ctx*> inst;
    hipStream_t stream = nullptr;       // caller's stream: every launch and copy
    hipStream_t cap = nullptr;          // private stream used only to capture graphs
    int seg_rows = 8;
    int mode = TEUK_BATCH_PER_ITERATION;   // the faster mode on every batch measured
    int ntiles = 0;                     // tiles per iteration at seg_rows
    int items = 0;                      // (strip, segment) items per iteration at seg_rows
    int max_tiles = 0;                  // at the smallest segment (allocation size)
    int waves = 0;                      // persistent waves per launch
    int resident_waves = 0;             // 8 per CU (two per SIMD at the kernel's register use)
    long long wait_limit = 0;
    int wall_khz = 1;                   // device wall clock rate (kHz) the wait limit is counted in
    teuk::BatchInstance* h_inst[2] = {nullptr, nullptr};   // pinned, alternate calls
    hipEvent_t h_inst_free[2] = {nullptr, nullptr};        // copy out of h_inst[k] finished
    int slot = 0;
    teuk::BatchInstance* d_inst = nullptr;
    int4* d_tiles = nullptr;
    int* d_item0 = nullptr;             // per instance: first item (per-iteration mode), + total
    std::vector<int> h_item0;           // host copy of d_item0
    std::vector<int> order;             // device table position -> instance (caller's index)
    std::vector<int> groups;            // per-iteration mode: first table position of each group, + count
    int* d_done = nullptr;
    unsigned long long* d_ticket = nullptr;
    int* d_abort = nullptr;
    std::vector<BatchGraph> graphs;
};

namespace {

// One tile per strip of 62 columns of each instance.
int tiles_for(const teuk_batch* b) {
    long total = 0;
    for (const teuk_ctx* c : b->inst) total += c->nstrips;
    return total > INT_MAX ? -1 : static_cast<int>(total);
}

void drop_graphs(teuk_batch* b) {
    for (auto& g : b->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    b->graphs.clear();
}

void free_batch(teuk_batch* b) {
    (void)hipStreamSynchronize(b->stream);
    drop_graphs(b);
    for (teuk_ctx* c : b->inst) teuk_detail::destroy_ctx(c);
    b->inst.clear();
    for (int k = 0; k < 2; ++k) {
        if (b->h_inst[k]) (void)hipHostFree(b->h_inst[k]);
        if (b->h_inst_free[k]) (void)hipEventDestroy(b->h_inst_free[k]);
    }
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;   // the device tables are the caller's workspace
}

// Byte offsets of the batch's own tables at the start of its workspace; the
// instances' workspaces follow from `first`, each `inst[k]` bytes long.
struct BatchLayout {
    size_t d_inst = 0, d_tiles = 0, d_item0 = 0, d_done = 0, d_ticket = 0, d_abort = 0, first = 0, total = 0;
    std::vector<size_t> inst;
};

std::string batch_layout(int32_t n, const teuk_grid_desc* descs, const teuk_ws_request* req, BatchLayout* L) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += (bytes + 255) / 256 * 256;
        return at;
    };
    long tiles = 0;
    L->inst.assign(static_cast<size_t>(n), 0);
    std::vector<size_t> sizes;
    for (int32_t k = 0; k < n; ++k) {
        const teuk_grid_desc* d = &descs[k];
        if (!(d->ko_eps >= 0.0 && d->ko_eps <= 1.0)) return "instance " + std::to_string(k) + ": need 0 <= ko_eps <= 1";
        teuk::Geometry G;
        std::string err = teuk::build_geometry(d->M, d->a, d->s, d->m, d->nr, d->nth, d->rs_min, d->rs_max, d->cfl,
                                               d->rs_extract, G);
        teuk_detail::WsLayout W;
        if (err.empty()) err = teuk_detail::ws_layout(G, (G.nr + 15) / 16 * 16, req, &W);
        if (!err.empty()) return "instance " + std::to_string(k) + ": " + err;
        L->inst[k] = W.total;
        tiles += (G.nr + 61) / 62;
        if (tiles > INT_MAX / 2) return "too many tiles in one batch";
    }
    L->d_inst = take(sizeof(teuk::BatchInstance) * static_cast<size_t>(n));
    L->d_tiles = take(sizeof(int4) * static_cast<size_t>(tiles));
    L->d_item0 = take(sizeof(int) * (static_cast<size_t>(n) + 1));
    L->d_done = take(sizeof(int) * static_cast<size_t>(tiles));
    L->d_ticket = take(sizeof(unsigned long long));
    L->d_abort = take(sizeof(int));
    L->first = off;
    for (size_t w : L->inst) take(w);
    L->total = off;
    return "";
}

// Theta segments per strip at segment length seg (the last takes up to
// seg + 2 rows, as in teuk_step_n).
int segments(const teuk_ctx* c, int seg) { return (c->G.nth - 3) / seg + 1; }

// Tile list of the persistent mode: instance-major, then strip; tile index =
// position in the list (also the index of its done counter).  The segment
// length only changes how each wave walks its strip.  Item offsets of the
// per-iteration mode: instance k owns items [item0[k], item0[k+1]), one per
// (strip, segment).
// Groups of the per-iteration mode.  When the batch's two state levels do
// not fit the last-level cache (256 MB on MI355X), the instances are packed
// into groups whose levels stay within kGroupLevelBytes (first fit, largest
// first; an instance larger than that is a group of its own), and each group
// is stepped through a whole chunk of iterations before the next: its two
// levels then stay in the cache over the chunk instead of streaming from
// HBM every iteration.  The device table holds the instances group by group
// (b->order), so that a group is a contiguous slice of it.  A batch that
// fits is one group in the caller's order: splitting it would only shorten
// its launches.
constexpr size_t kLastLevelCacheBytes = size_t(256) << 20;
constexpr size_t kGroupLevelBytes = size_t(96) << 20;

size_t level_bytes(const teuk_ctx* c) { return 2 * sizeof(double2) * static_cast<size_t>(c->ld) * c->G.nth; }

void set_batch_groups(teuk_batch* b) {
    const int n = static_cast<int>(b->inst.size());
    b->order.resize(n);
    for (int k = 0; k < n; ++k) b->order[k] = k;
    b->groups.assign({0, n});
    size_t total = 0;
    for (const teuk_ctx* c : b->inst) total += level_bytes(c);
    if (2 * total <= kLastLevelCacheBytes) return;
    std::vector<int> by_size(b->order);
    std::stable_sort(by_size.begin(), by_size.end(),
                     [&](int x, int y) { return level_bytes(b->inst[x]) > level_bytes(b->inst[y]); });
    std::vector<std::vector<int>> bins;
    std::vector<size_t> fill;
    for (int k : by_size) {
        const size_t sz = level_bytes(b->inst[k]);
        size_t at = bins.size();
        for (size_t g = 0; g < bins.size(); ++g)
            if (fill[g] + sz <= kGroupLevelBytes) {
                at = g;
                break;
            }
        if (at == bins.size()) {
            bins.emplace_back();
            fill.push_back(0);
        }
        bins[at].push_back(k);
        fill[at] += sz;
    }
    b->order.clear();
    b->groups.clear();
    for (auto& bin : bins) {
        std::sort(bin.begin(), bin.end());
        b->groups.push_back(static_cast<int>(b->order.size()));
        b->order.insert(b->order.end(), bin.begin(), bin.end());
    }
    b->groups.push_back(n);
}

int set_batch_tiles(teuk_batch* b, int seg) {
    std::vector<int4> tiles;
    tiles.reserve(b->max_tiles);
    std::vector<int> item0;
    long long items = 0;
    for (size_t k = 0; k < b->inst.size(); ++k) {   // k: position in the device table
        teuk_ctx* c = b->inst[b->order[k]];
        for (int s = 0; s < c->nstrips; ++s)
            tiles.push_back(make_int4(static_cast<int>(k), s, 0, static_cast<int>(tiles.size())));
        item0.push_back(static_cast<int>(items));
        items += static_cast<long long>(c->nstrips) * segments(c, seg);
        if (items > INT_MAX - 3) return fail(TEUK_EINVAL, "too many work items in one batch");
    }
    item0.push_back(static_cast<int>(items));
    b->h_item0 = item0;
    HIP_TRY(hipMemcpy(b->d_tiles, tiles.data(), sizeof(int4) * tiles.size(), hipMemcpyHostToDevice),
            "batch tiles");
    HIP_TRY(hipMemcpy(b->d_item0, item0.data(), sizeof(int) * item0.size(), hipMemcpyHostToDevice),
            "batch item offsets");
    b->items = static_cast<int>(items);
    b->seg_rows = seg;
    b->ntiles = static_cast<int>(tiles.size());
    b->waves = std::max(1, std::min(b->resident_waves, b->ntiles));
    return TEUK_OK;
}

// Source windows of a launch's first iteration in an instance's tables (all
// null without a source).
struct SourceView {
    const double2* fh = nullptr;
    const double2* fn = nullptr;
    const int4* org = nullptr;
    int win_r = 0, win_t = 0;
};

// Instance table of the next launch: static fields plus each instance's
// current level, waveform pointer (row offset `row` of its buffer) and
// source windows.  Alternates between two pinned buffers; a buffer is
// rewritten only after its previous copy has finished.
int upload_instances(teuk_batch* b, void* const* waveforms, int64_t row, const std::vector<SourceView>& src) {
    const int k = b->slot;
    b->slot ^= 1;
    HIP_TRY(hipEventSynchronize(b->h_inst_free[k]), "batch table reuse");
    teuk::BatchInstance* h = b->h_inst[k];
    int tile0 = 0;
    for (size_t j = 0; j < b->inst.size(); ++j) {   // j: position in the device table
        const int k_inst = b->order[j];
        const teuk_ctx* c = b->inst[k_inst];
        const teuk::Geometry& G = c->G;
        teuk::BatchInstance& I = h[j];
        for (int l = 0; l < 2; ++l)
            for (int f = 0; f < 2; ++f) I.plane[l][f] = c->plane[l][f];
        I.rnode = c->d_rnode;
        I.rhalf = c->d_rhalf;
        I.rows = c->d_rows;
        I.nr = G.nr;
        I.nth = G.nth;
        I.ld = c->ld;
        I.rpitch = G.nr;
        I.nstrips = c->nstrips;
        I.nseg = segments(c, b->seg_rows);
        I.dt = G.dt;
        I.inv_hr = 1.0 / G.h_r;
        I.ko_c = c->ko_c;
        I.even = (std::abs(G.m) % 2 == 0);
        I.kerr = (G.a != 0.0);
        I.i_ext = G.i_ext;
        I.cur = c->cur;
        I.tile0 = tile0;
        I.wave = (waveforms && waveforms[k_inst]) ? static_cast<double2*>(waveforms[k_inst]) + row * G.nth : nullptr;
        I.fh = src[k_inst].fh;
        I.fn = src[k_inst].fn;
        I.org = src[k_inst].org;
        I.win_r = src[k_inst].win_r;
        I.win_t = src[k_inst].win_t;
        tile0 += I.nstrips;
    }
    HIP_TRY(hipMemcpyAsync(b->d_inst, h, sizeof(teuk::BatchInstance) * b->inst.size(), hipMemcpyHostToDevice,
                           b->stream),
            "batch table upload");
    HIP_TRY(hipEventRecord(b->h_inst_free[k], b->stream), "batch table event");
    return TEUK_OK;
}

// Captured graph for (rounds, seg_rows): reset the counters, then the
// persistent launch.  Kept in a small cache.
int graph_for(teuk_batch* b, int64_t rounds, hipGraphExec_t* out) {
    for (auto& g : b->graphs)
        if (g.rounds == rounds && g.seg == b->seg_rows) {
            *out = g.exec;
            return TEUK_OK;
        }
    if (static_cast<int>(b->graphs.size()) == kGraphCache) {
        (void)hipGraphExecDestroy(b->graphs.front().exec);
        (void)hipGraphDestroy(b->graphs.front().graph);
        b->graphs.erase(b->graphs.begin());
    }
    teuk::BatchParams B;
    B.inst = b->d_inst;
    B.tiles = b->d_tiles;
    B.ntiles = b->ntiles;
    B.rounds = static_cast<int>(rounds);
    B.ticket = b->d_ticket;
    B.done = b->d_done;
    B.abort = b->d_abort;
    B.wait_limit = b->wait_limit;
    BatchGraph g;
    g.rounds = rounds;
    g.seg = b->seg_rows;
    HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal), "batch capture begin");
    hipError_t e1 = teuk::launch_batch_reset(B, b->cap);
    hipError_t e2 = (e1 == hipSuccess) ? teuk::launch_batch(B, b->seg_rows, b->waves, b->cap) : e1;
    hipError_t e3 = hipStreamEndCapture(b->cap, &g.graph);
    if (e2 != hipSuccess) {
        if (g.graph) (void)hipGraphDestroy(g.graph);
        return hip_fail(e2, "batch capture");
    }
    if (e3 != hipSuccess) return hip_fail(e3, "batch capture end");
    hipError_t e4 = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
    if (e4 != hipSuccess) {
        (void)hipGraphDestroy(g.graph);
        return hip_fail(e4, "batch graph instantiate");
    }
    b->graphs.push_back(g);
    *out = g.exec;
    return TEUK_OK;
}

int check_batch(const teuk_batch* b) {
    if (b == nullptr) return fail(TEUK_EINVAL, "null batch");
    return TEUK_OK;
}

}  // namespace

extern "C" {

int teuk_batch_workspace_size(int32_t n, const teuk_grid_desc* descs, const teuk_ws_request* req, size_t* bytes) {
    if (bytes == nullptr || descs == nullptr) return fail(TEUK_EINVAL, "null descriptors or output");
    *bytes = 0;
    if (n < 1) return fail(TEUK_EINVAL, "a batch needs at least one instance");
    BatchLayout L;
    const std::string err = batch_layout(n, descs, req, &L);
    if (!err.empty()) return fail(TEUK_EINVAL, err);
    *bytes = L.total;
    return TEUK_OK;
}

int teuk_batch_create(int32_t n, const teuk_grid_desc* descs, const teuk_ws_request* req, void* hip_stream,
                      void* ws, size_t ws_bytes, teuk_batch** out) {
    if (out == nullptr || descs == nullptr) return fail(TEUK_EINVAL, "null descriptors or output");
    *out = nullptr;
    if (n < 1) return fail(TEUK_EINVAL, "a batch needs at least one instance");
    if (ws == nullptr || reinterpret_cast<uintptr_t>(ws) % 256 != 0)
        return fail(TEUK_EINVAL, "the batch workspace must be a 256-byte aligned device pointer");
    BatchLayout L;
    const std::string err = batch_layout(n, descs, req, &L);
    if (!err.empty()) return fail(TEUK_EINVAL, err);
    if (ws_bytes < L.total)
        return fail(TEUK_ENOMEM, "batch workspace of " + std::to_string(ws_bytes) + " bytes, need " +
                                     std::to_string(L.total));
    teuk_batch* b = new (std::nothrow) teuk_batch();
    if (b == nullptr) return fail(TEUK_ENOMEM, "host allocation failed");
    b->stream = static_cast<hipStream_t>(hip_stream);
    char* base = static_cast<char*>(ws);
    size_t off = L.first;
    for (int32_t k = 0; k < n; ++k) {
        teuk_ctx* c = nullptr;
        if (int rc = teuk_detail::make_ctx(&descs[k], req, hip_stream, base + off, L.inst[k], &c)) {
            const std::string msg = "instance " + std::to_string(k) + ": " + teuk_detail::g_last_error;
            free_batch(b);
            return fail(rc, msg);
        }
        off += (L.inst[k] + 255) / 256 * 256;
        c->in_batch = true;
        b->inst.push_back(c);
    }
    b->max_tiles = tiles_for(b);
    if (b->max_tiles < 0) {
        free_batch(b);
        return fail(TEUK_EINVAL, "too many tiles in one batch");
    }
    b->d_inst = reinterpret_cast<teuk::BatchInstance*>(base + L.d_inst);
    b->d_tiles = reinterpret_cast<int4*>(base + L.d_tiles);
    b->d_item0 = reinterpret_cast<int*>(base + L.d_item0);
    b->d_done = reinterpret_cast<int*>(base + L.d_done);
    b->d_ticket = reinterpret_cast<unsigned long long*>(base + L.d_ticket);
    b->d_abort = reinterpret_cast<int*>(base + L.d_abort);
    int dev = 0, cus = 0, khz = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    for (int k = 0; k < 2 && e == hipSuccess; ++k) {
        e = hipHostMalloc(reinterpret_cast<void**>(&b->h_inst[k]), sizeof(teuk::BatchInstance) * n);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b->h_inst_free[k], hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventRecord(b->h_inst_free[k], b->stream);
    }
    if (e == hipSuccess) e = teuk::launch_zero(b->d_abort, sizeof(int), b->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess) {
        free_batch(b);
        return hip_fail(e, "batch setup");
    }
    b->resident_waves = 8 * std::max(cus, 1);
    b->wall_khz = std::max(khz, 1);
    b->wait_limit = static_cast<long long>(kWaitLimitSeconds * 1e3 * b->wall_khz);
    const int seg = 16;   // long segments, fewest halo rows (the autotuner measures 4, 8 and 16)
    set_batch_groups(b);
    if (int rc = set_batch_tiles(b, seg)) {
        const std::string msg = teuk_detail::g_last_error;
        free_batch(b);
        return fail(rc, msg);
    }
    *out = b;
    return TEUK_OK;
}

int teuk_batch_destroy(teuk_batch* b) {
    if (b == nullptr) return TEUK_OK;
    free_batch(b);
    return TEUK_OK;
}

int teuk_batch_instance(teuk_batch* b, int32_t k, teuk_ctx** out) {
    if (int rc = check_batch(b)) return rc;
    if (out == nullptr) return fail(TEUK_EINVAL, "null output");
    if (k < 0 || k >= static_cast<int32_t>(b->inst.size())) return fail(TEUK_EINVAL, "instance index out of range");
    *out = b->inst[k];
    return TEUK_OK;
}

int teuk_batch_set_tuning(teuk_batch* b, int32_t seg_rows) {
    if (int rc = check_batch(b)) return rc;
    if (!teuk::valid_segment_rows(seg_rows)) return fail(TEUK_EINVAL, "seg_rows must be 4, 8 or 16");
    HIP_TRY(hipStreamSynchronize(b->stream), "batch tuning");
    return set_batch_tiles(b, seg_rows);
}

int teuk_batch_get_tuning(const teuk_batch* b, int32_t* seg_rows) {
    if (int rc = check_batch(b)) return rc;
    if (seg_rows == nullptr) return fail(TEUK_EINVAL, "null output");
    *seg_rows = b->seg_rows;
    return TEUK_OK;
}

int teuk_batch_set_mode(teuk_batch* b, int32_t mode) {
    if (int rc = check_batch(b)) return rc;
    if (mode != TEUK_BATCH_PERSISTENT && mode != TEUK_BATCH_PER_ITERATION)
        return fail(TEUK_EINVAL, "mode must be TEUK_BATCH_PERSISTENT or TEUK_BATCH_PER_ITERATION");
    b->mode = mode;
    return TEUK_OK;
}

int teuk_batch_get_mode(const teuk_batch* b, int32_t* mode) {
    if (int rc = check_batch(b)) return rc;
    if (mode == nullptr) return fail(TEUK_EINVAL, "null output");
    *mode = b->mode;
    return TEUK_OK;
}

int teuk_batch_get_groups(const teuk_batch* b, int32_t* ngroups, int32_t* first, int32_t* order) {
    if (int rc = check_batch(b)) return rc;
    if (ngroups == nullptr) return fail(TEUK_EINVAL, "null output");
    const int ng = static_cast<int>(b->groups.size()) - 1;
    *ngroups = ng;
    if (first != nullptr)
        for (int g = 0; g <= ng; ++g) first[g] = b->groups[g];
    if (order != nullptr)
        for (size_t k = 0; k < b->order.size(); ++k) order[k] = b->order[k];
    return TEUK_OK;
}

int teuk_batch_step_n(teuk_batch* b, int64_t nsteps, void* const* waveforms) {
    if (int rc = check_batch(b)) return rc;
    if (nsteps < 0 || nsteps > INT_MAX) return fail(TEUK_EINVAL, "nsteps out of range");
    if (nsteps == 0) return TEUK_OK;
    bool any_src = false;
    for (size_t k = 0; k < b->inst.size(); ++k) {
        const teuk_ctx* c = b->inst[k];
        if (!c->has_src) continue;
        any_src = true;
        if (2 * (c->steps_done + nsteps - 1) + 1 >= c->nsamples)
            return fail(TEUK_ESTATE, "instance " + std::to_string(k) + ": orbit has too few samples for the "
                                                                     "requested steps");
    }
    // With sources the iterations go in chunks of at most one source batch:
    // each chunk starts with the compact source pass of every instance that
    // has a source (as teuk_step_n), then the chunk's launch(es).
    const int64_t chunk_max = any_src ? kSourceBatch : nsteps;
    if (static_cast<unsigned long long>(chunk_max) * static_cast<unsigned long long>(b->ntiles) >= (1ull << 62))
        return fail(TEUK_EINVAL, "too many work items in one launch");
    std::vector<SourceView> src(b->inst.size());
    for (int64_t done = 0; done < nsteps;) {
        const int64_t len = std::min(nsteps - done, chunk_max);
        for (size_t k = 0; k < b->inst.size(); ++k) {
            teuk_ctx* c = b->inst[k];
            if (!c->has_src) continue;
            const int64_t n = c->steps_done;
            const int64_t span = (c->nsamples - 2) / 2 - n + 1;   // iterations the orbit still supports
            size_t slot = 0;
            if (int rc = teuk_detail::ensure_source(c, n, c->amplitude, false, span, &slot)) return rc;
            if (static_cast<int64_t>(slot) + len > c->batch_len) {   // the chunk must fit one batch
                c->batch_n0 = -1;                                     // (empty: start a new one at n)
                c->batch_len = 0;
                if (int rc = teuk_detail::ensure_source(c, n, c->amplitude, false, span, &slot)) return rc;
            }
            const size_t wsz = static_cast<size_t>(c->win_r) * c->win_t;
            src[k].fh = c->d_fh + slot * wsz;
            src[k].fn = c->d_fn + slot * wsz;
            src[k].org = c->d_org + slot;
            src[k].win_r = c->win_r;
            src[k].win_t = c->win_t;
        }
        if (b->mode == TEUK_BATCH_PER_ITERATION) {
            if (int rc = upload_instances(b, waveforms, done, src)) return rc;
            // group by group, each through the whole chunk: one launch per
            // iteration over the group's instances
            for (size_t g = 0; g + 1 < b->groups.size(); ++g) {
                const int k0 = b->groups[g], k1 = b->groups[g + 1];
                const int base = b->h_item0[k0], items = b->h_item0[k1] - base;
                for (int64_t n = 0; n < len; ++n)
                    HIP_TRY(teuk::launch_batch_iteration(b->d_inst + k0, b->d_item0 + k0, k1 - k0, base, items,
                                                         static_cast<int>(n), b->seg_rows, b->stream),
                            "batch iteration launch");
            }
        } else {
            hipGraphExec_t exec = nullptr;
            if (int rc = graph_for(b, len, &exec)) return rc;
            if (int rc = upload_instances(b, waveforms, done, src)) return rc;
            HIP_TRY(hipGraphLaunch(exec, b->stream), "batch graph launch");
        }
        for (teuk_ctx* c : b->inst) {
            c->cur ^= static_cast<int>(len & 1);
            c->steps_done += len;
        }
        done += len;
    }
    return TEUK_OK;
}

int teuk_batch_set_wait_limit(teuk_batch* b, double seconds) {
    if (int rc = check_batch(b)) return rc;
    if (!(seconds >= 0.0 && seconds <= 3600.0)) return fail(TEUK_EINVAL, "wait limit must be in [0, 3600] s");
    HIP_TRY(hipStreamSynchronize(b->stream), "batch wait limit");
    b->wait_limit = static_cast<long long>(seconds * 1e3 * b->wall_khz);
    drop_graphs(b);   // the limit is a kernel argument of the captured launches
    return TEUK_OK;
}

int teuk_batch_abort(teuk_batch* b) {
    if (int rc = check_batch(b)) return rc;
    HIP_TRY(hipMemsetD32Async(reinterpret_cast<hipDeviceptr_t>(b->d_abort), 1, 1, b->stream), "batch abort");
    return TEUK_OK;
}

int teuk_batch_sync(teuk_batch* b) {
    if (int rc = check_batch(b)) return rc;
    HIP_TRY(hipStreamSynchronize(b->stream), "batch sync");
    int flag = 0;
    HIP_TRY(hipMemcpy(&flag, b->d_abort, sizeof(int), hipMemcpyDeviceToHost), "batch abort flag");
    if (flag != 0) {
        HIP_TRY(hipMemset(b->d_abort, 0, sizeof(int)), "batch abort flag clear");
        return fail(TEUK_EDEVICE, "batched launch aborted (a dependency wait exceeded its limit, or "
                                  "teuk_batch_abort); instance states are invalid");
    }
    return TEUK_OK;
}

int teuk_batch_autotune(teuk_batch* b, const char* cache_path, teuk_tune_entry* table, int32_t capacity,
                        int32_t* count) {
    if (int rc = check_batch(b)) return rc;
    if (count != nullptr) *count = 0;
    if (table != nullptr && capacity < 0) return fail(TEUK_EINVAL, "negative table capacity");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "autotune device");
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev), "autotune device properties");
    std::string arch = prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
    // key: architecture, the instance shapes, and the kernel sources
    unsigned long long h = 1469598103934665603ull;   // FNV-1a over the shapes
    auto mix = [&](long long v) {
        for (int k = 0; k < 8; ++k) {
            h ^= static_cast<unsigned long long>((v >> (8 * k)) & 0xff);
            h *= 1099511628211ull;
        }
    };
    for (const teuk_ctx* c : b->inst) {
        mix(c->G.nr);
        mix(c->G.nth);
        mix(c->G.a != 0.0);
        mix(c->ko_c != 0.0);
    }
    char keybuf[256];
    std::snprintf(keybuf, sizeof(keybuf), "%s batch n=%zu shapes=%016llx src=%s", arch.c_str(), b->inst.size(), h,
                  TEUK_SOURCE_HASH);
    const std::string key = keybuf;
    auto emit = [&](const std::vector<teuk_tune_entry>& v) {
        int32_t w = 0;
        if (table != nullptr)
            for (const auto& e : v)
                if (w < capacity) table[w++] = e;
        if (count != nullptr) *count = w;
    };
    if (cache_path != nullptr) {
        std::ifstream f(cache_path);
        std::string line;
        bool found = false;
        teuk_tune_entry hit{};
        while (f && std::getline(f, line)) {
            std::istringstream ls(line);
            std::string k, seg, kk, us, md;
            if (!std::getline(ls, k, '\t') || !std::getline(ls, seg, '\t') || !std::getline(ls, kk, '\t') ||
                !std::getline(ls, us, '\t') || !std::getline(ls, md, '\t'))
                continue;
            if (k != key) continue;
            const int s = std::atoi(seg.c_str());
            const int m = std::atoi(md.c_str());
            if (teuk::valid_segment_rows(s) && std::atoi(kk.c_str()) == 1 &&
                (m == TEUK_BATCH_PERSISTENT || m == TEUK_BATCH_PER_ITERATION)) {
                hit = {s, 1, m, std::atof(us.c_str())};
                found = true;
            }
        }
        if (found) {
            if (hit.seg_rows != b->seg_rows)
                if (int rc = teuk_batch_set_tuning(b, hit.seg_rows)) return rc;
            b->mode = hit.batch_mode;
            emit({hit});
            return TEUK_OK;
        }
    }

    // save every instance's current level, time each variant, restore
    const int seg0 = b->seg_rows, mode0 = b->mode;
    // every instance's current level goes to host memory for the trials
    std::vector<std::vector<double2>> save;
    hipError_t e = hipSuccess;
    HIP_TRY(hipStreamSynchronize(b->stream), "batch autotune sync");
    try {
        for (teuk_ctx* c : b->inst) {
            const size_t bytes = sizeof(double2) * static_cast<size_t>(c->ld) * c->G.nth;
            for (int f = 0; f < 2; ++f) {
                save.emplace_back(bytes / sizeof(double2));
                HIP_TRY(hipMemcpy(save.back().data(), c->plane[c->cur][f], bytes, hipMemcpyDeviceToHost),
                        "batch autotune save");
            }
        }
    } catch (const std::bad_alloc&) {
        return fail(TEUK_ENOMEM, "batch autotune: host copy of the states");
    }
    // sources are detached while timing (the compact source pass is a small
    // part of an iteration, and the orbits need not extend past the call)
    std::vector<int> cur0;
    std::vector<int64_t> steps_done0;
    std::vector<char> src0;
    for (teuk_ctx* c : b->inst) {
        cur0.push_back(c->cur);
        steps_done0.push_back(c->steps_done);
        src0.push_back(c->has_src ? 1 : 0);
        c->has_src = false;
    }
    auto restore = [&]() {
        (void)hipStreamSynchronize(b->stream);
        for (size_t k = 0; k < b->inst.size(); ++k) {
            teuk_ctx* c = b->inst[k];
            const size_t bytes = sizeof(double2) * static_cast<size_t>(c->ld) * c->G.nth;
            c->cur = cur0[k];
            c->steps_done = steps_done0[k];
            c->has_src = src0[k] != 0;
            for (int f = 0; f < 2; ++f)
                (void)hipMemcpy(c->plane[c->cur][f], save[2 * k + f].data(), bytes, hipMemcpyHostToDevice);
        }
    };
    hipEvent_t ev[2] = {nullptr, nullptr};
    e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    if (e != hipSuccess) {
        restore();
        return hip_fail(e, "batch autotune events");
    }
    std::vector<teuk_tune_entry> cand;
    for (int mode : {TEUK_BATCH_PERSISTENT, TEUK_BATCH_PER_ITERATION})
        for (int seg : teuk::kSegVariants) cand.push_back({seg, 1, mode, 0.0});
    constexpr int kRounds = 8, kReps = 3;
    int rc = TEUK_OK;
    for (auto& t : cand) {
        rc = teuk_batch_set_tuning(b, t.seg_rows);
        if (rc == TEUK_OK) rc = teuk_batch_set_mode(b, t.batch_mode);
        if (rc == TEUK_OK) rc = teuk_batch_step_n(b, kRounds, nullptr);   // warm-up (and capture)
        double best = 1e300;
        for (int r = 0; rc == TEUK_OK && r < kReps; ++r) {
            float ms = 0.0f;
            e = hipEventRecord(ev[0], b->stream);
            if (e == hipSuccess) rc = teuk_batch_step_n(b, kRounds, nullptr);
            if (e == hipSuccess && rc == TEUK_OK) e = hipEventRecord(ev[1], b->stream);
            if (e == hipSuccess && rc == TEUK_OK) e = hipEventSynchronize(ev[1]);
            if (e == hipSuccess && rc == TEUK_OK) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
            if (e != hipSuccess && rc == TEUK_OK) rc = hip_fail(e, "batch autotune timing");
            best = std::min(best, 1e3 * static_cast<double>(ms) / kRounds);
        }
        if (rc == TEUK_OK) rc = teuk_batch_sync(b);
        if (rc != TEUK_OK) break;
        t.us_per_iteration = best;
    }
    const std::string msg = teuk_detail::g_last_error;
    restore();
    for (auto& x : ev) (void)hipEventDestroy(x);
    if (rc != TEUK_OK) {
        (void)teuk_batch_set_tuning(b, seg0);
        b->mode = mode0;
        return fail(rc, msg);
    }
    std::stable_sort(cand.begin(), cand.end(), [](const teuk_tune_entry& x, const teuk_tune_entry& y) {
        return x.us_per_iteration < y.us_per_iteration;
    });
    if (int r2 = teuk_batch_set_tuning(b, cand[0].seg_rows)) return r2;
    b->mode = cand[0].batch_mode;
    emit(cand);
    if (cache_path != nullptr) {
        std::ofstream f(cache_path, std::ios::app);
        char line[512];
        std::snprintf(line, sizeof(line), "%s\t%d\t%d\t%.4f\t%d\n", key.c_str(), cand[0].seg_rows, 1,
                      cand[0].us_per_iteration, cand[0].batch_mode);
        if (!(f << line)) return fail(TEUK_EINVAL, std::string("cannot append to tuning cache ") + cache_path);
    }
    return TEUK_OK;
}

}  // extern "C"
