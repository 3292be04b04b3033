// C ABI of the engine (declared in include/teuk.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <mutex>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/teuk.h"
#include "ctx.h"
#include "geometry.h"
#include "item_order.h"
#include "kernels.h"
#include "revolve.h"

using teuk::Geometry;
using teuk::ThetaRow;

namespace teuk_detail {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

int hip_fail(hipError_t e, const char* what) {
    return fail(TEUK_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

}  // namespace teuk_detail

using teuk_detail::ensure_source;
using teuk_detail::fail;
using teuk_detail::g_last_error;
using teuk_detail::hip_fail;
using teuk_detail::kSourceBatch;

namespace {

#ifndef TEUK_SOURCE_HASH
#define TEUK_SOURCE_HASH "unversioned"
#endif

constexpr int kPartSteps = 64;      // adjoint iterations whose dL/dA partials are reduced together

}  // namespace

namespace {

void free_source(teuk_ctx* c) {
    c->d_orbit = nullptr;          // the caller's buffer
    c->h_orbit.clear();
    c->has_src = false;
    c->batch_n0 = -1;
    c->batch_len = 0;
}

// Sum the recorded event pairs into the context's totals (synchronizes).
int flush_timing(teuk_ctx* c) {
    if (c->ev_used == 0) return TEUK_OK;
    HIP_TRY(hipEventSynchronize(c->ev_stop[c->ev_used - 1]), "timing sync");
    for (size_t k = 0; k < c->ev_used; ++k) {
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, c->ev_start[k], c->ev_stop[k]), "timing elapsed");
        c->timed_ms += ms;
        c->timed_launches += 1;
    }
    c->ev_used = 0;
    return TEUK_OK;
}

void destroy_events(teuk_ctx* c) {
    for (auto e : c->ev_start) (void)hipEventDestroy(e);
    for (auto e : c->ev_stop) (void)hipEventDestroy(e);
    c->ev_start.clear();
    c->ev_stop.clear();
    c->ev_used = 0;
}

constexpr size_t kTimingPool = 2048;

void reset_adjoint(teuk_ctx* c) { c->adj_clock = -1; }

void reset_ckpt(teuk_ctx* c) {
    c->snaps = nullptr;
    c->seg_buf = nullptr;
    c->d_ls = c->d_ls_part = nullptr;
    c->ckpt_valid = false;
}

// Devices whose static workspace a live context holds (teuk_init_grid_static).
std::mutex g_static_mutex;
std::vector<int> g_static_busy;

// A context made on the library's static workspace gives it back.
void release_static_workspace(teuk_ctx* c) {
    if (c->static_dev < 0) return;
    std::lock_guard<std::mutex> lock(g_static_mutex);
    g_static_busy.erase(std::remove(g_static_busy.begin(), g_static_busy.end(), c->static_dev), g_static_busy.end());
    c->static_dev = -1;
}

void release_host_state(teuk_ctx* c) {
    destroy_events(c);
    reset_ckpt(c);
    reset_adjoint(c);
    free_source(c);
}

}  // namespace

void teuk_detail::destroy_ctx(teuk_ctx* c) {
    (void)hipStreamSynchronize(c->stream);
    release_host_state(c);
    release_static_workspace(c);
    delete c;
}

namespace {

int check_ctx(const teuk_ctx* c) {
    if (c == nullptr) return fail(TEUK_EINVAL, "null context");
    return TEUK_OK;
}

}  // namespace

// Forward stepping fills [n, n + nb); the reverse sweep fills [n - nb + 1, n].
int teuk_detail::ensure_source(teuk_ctx* c, int64_t n, double amp, bool backward, int64_t span, size_t* slot) {
    if (!(n >= c->batch_n0 && n < c->batch_n0 + c->batch_len && amp == c->batch_amp)) {
        const int nb = static_cast<int>(span < kSourceBatch ? span : kSourceBatch);
        const int64_t n0 = backward ? n - nb + 1 : n;
        const Geometry& G = c->G;
        teuk::SourceParams S;
        S.n0 = static_cast<int>(n0);
        S.org = c->d_org;
        S.win_r = c->win_r;
        S.win_t = c->win_t;
        S.orbit = c->d_orbit;
        S.amplitude = amp;
        S.sig_r = c->sig_r;
        S.sig_th = c->sig_th;
        S.cut = c->cut;
        S.rs_min = G.rs_min;
        S.h_r = G.h_r;
        S.h_th = G.h_th;
        S.m = G.m;
        S.nr = G.nr;
        S.nth = G.nth;
        S.rnode_rs = c->d_rnode + static_cast<size_t>(teuk::RF_RS) * G.nr;
        S.rhalf_rs = c->d_rhalf + static_cast<size_t>(teuk::RF_RS) * G.nr;
        S.rows = c->d_rows;
        S.fh = c->d_fh;
        S.fn = c->d_fn;
        HIP_TRY(teuk::launch_source_pass(S, nb, c->stream), "source pass");
        c->batch_n0 = n0;
        c->batch_len = nb;
        c->batch_amp = amp;
    }
    *slot = static_cast<size_t>(n - c->batch_n0);
    return TEUK_OK;
}

namespace {

void set_adjoint_segment(teuk_ctx* c, int seg) {
    c->adj_seg_rows = seg;
    c->adj_nseg = (c->G.nth - 3) / seg + 1;
}

void set_tuning_fields(teuk_ctx* c, int seg, int k) {
    c->seg_rows = seg;
    c->k_steps = k;
    c->nseg = (c->G.nth - 3) / seg + 1;
    const int w = teuk::block_strip_width(k);
    c->bstrips = (c->G.nr + w - 1) / w;
}

// The adjoint's work items (strip x segment) whose output rows and columns
// may meet the source windows of forward iteration m.  The origins are
// computed as the source pass computes them, from the host's copy of the
// same orbit samples, and widened by 2 cells against any difference in
// rounding; the kernel still tests every wave itself.  ns or ng is 0 when
// no item can meet them.
void source_items(const teuk_ctx* c, int64_t m, int seg_rows, int nseg, int& s0, int& ns, int& g0, int& ng,
                  int& row_lo, int& row_hi) {
    const Geometry& G = c->G;
    const double* sh = c->h_orbit.data() + 3 * static_cast<size_t>(2 * m);
    const double* sn = c->h_orbit.data() + 3 * static_cast<size_t>(2 * m + 1);
    const double Rr = c->cut * c->sig_r, Rt = c->cut * c->sig_th;
    auto idx = [](double v) { return static_cast<int>(std::fmin(std::fmax(std::floor(v), -1e8), 1e8)); };
    const int cx = idx((sh[0] - Rr - (G.rs_min + 0.5 * G.h_r)) / G.h_r);
    const int ry = idx((sh[1] - Rt) / G.h_th);
    const int cz = idx((sn[0] - Rr - G.rs_min) / G.h_r);
    const int rw = idx((sn[1] - Rt) / G.h_th);
    const int c_lo = std::min(cx, cz) - 2, c_hi = std::max(cx, cz) + c->win_r + 2;   // columns [c_lo, c_hi)
    const int r_lo = std::min(ry, rw) - 2, r_hi = std::max(ry, rw) + c->win_t + 2;   // rows [r_lo, r_hi)
    int slo = -1, shi = -1, glo = -1, ghi = -1;
    for (int s = 0; s < c->nstrips; ++s) {
        const int i0 = 62 * s - 1;   // the wave's 64 columns i0 .. i0 + 63
        if (c_lo <= i0 + 63 && i0 < c_hi) {
            if (slo < 0) slo = s;
            shi = s;
        }
    }
    for (int g = 0; g < nseg; ++g) {
        const int jlo = g * seg_rows, jhi = (g == nseg - 1) ? G.nth : jlo + seg_rows;
        if (r_lo <= jhi - 1 && jlo < r_hi) {
            if (glo < 0) glo = g;
            ghi = g;
        }
    }
    s0 = std::max(slo, 0);
    g0 = std::max(glo, 0);
    ns = slo < 0 ? 0 : shi - slo + 1;
    ng = glo < 0 ? 0 : ghi - glo + 1;
    row_lo = r_lo;
    row_hi = r_hi;
}

int flush_partials(teuk_ctx* c) {
    if (c->part_filled == 0) return TEUK_OK;
    HIP_TRY(teuk::launch_reduce_partials(c->d_dA_part, c->part_items * c->part_filled, c->d_dA_blk, c->d_dA,
                                         c->stream),
            "dA reduction");
    c->part_filled = 0;
    return TEUK_OK;
}

int row_pitch(int nr) { return (nr + 15) / 16 * 16; }

}  // namespace

std::string teuk_detail::ws_layout(const Geometry& G, int ld, const teuk_ws_request* req, WsLayout* L) {
    *L = WsLayout{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += (bytes + 255) / 256 * 256;
        return at;
    };
    const size_t plane_bytes = sizeof(double2) * static_cast<size_t>(ld) * G.nth;
    L->planes = take(4 * plane_bytes);
    const size_t rbytes = sizeof(double) * teuk::RF_COUNT * static_cast<size_t>(G.nr);
    L->rnode = take(rbytes);
    L->rhalf = take(rbytes);
    L->rows = take(sizeof(ThetaRow) * G.nth);
    L->flag = take(sizeof(int));
    if (req != nullptr && (req->sigma_r_cells != 0.0 || req->sigma_th_cells != 0.0 || req->cutoff_sigmas != 0.0)) {
        if (!(req->sigma_r_cells > 0.0 && req->sigma_th_cells > 0.0 && req->cutoff_sigmas > 0.0))
            return "source footprint: widths and cutoff must all be positive (or all 0 for no source)";
        const double wr = std::ceil(2.0 * req->cutoff_sigmas * req->sigma_r_cells) + 2.0;
        const double wt = std::ceil(2.0 * req->cutoff_sigmas * req->sigma_th_cells) + 2.0;
        if (!(wr <= 4096.0 && wt <= 4096.0)) return "source footprint wider than 4096 cells";
        L->win_r_cap = static_cast<int>(wr);
        L->win_t_cap = static_cast<int>(wt);
        const size_t tbytes = sizeof(double2) * static_cast<size_t>(L->win_r_cap) * L->win_t_cap * kSourceBatch;
        L->fh = take(tbytes);
        L->fn = take(tbytes);
        L->org = take(sizeof(int4) * kSourceBatch);
    }
    if (req != nullptr && req->adjoint != 0) {
        L->adjoint = true;
        const int nstrips = (G.nr + 61) / 62;
        const size_t max_items = static_cast<size_t>(nstrips) * ((G.nth - 3) / 4 + 1);
        L->adj = take(4 * plane_bytes);
        L->dA = take(sizeof(double));
        L->dA_part = take(sizeof(double) * max_items * kPartSteps);
        L->dA_blk = take(sizeof(double) * teuk::reduce_partials_blocks(static_cast<int>(max_items * kPartSteps)));
    }
    L->total = off;
    return "";
}

int teuk_detail::make_ctx(const teuk_grid_desc* d, const teuk_ws_request* req, void* hip_stream, void* ws,
                          size_t ws_bytes, teuk_ctx** out) {
    if (d == nullptr || out == nullptr) return fail(TEUK_EINVAL, "null descriptor or output");
    *out = nullptr;
    if (!(d->ko_eps >= 0.0 && d->ko_eps <= 1.0)) return fail(TEUK_EINVAL, "need 0 <= ko_eps <= 1");
    if (ws == nullptr) return fail(TEUK_EINVAL, "null workspace");
    if (reinterpret_cast<uintptr_t>(ws) % 256 != 0) return fail(TEUK_EINVAL, "workspace must be 256-byte aligned");
    teuk_ctx* c = new (std::nothrow) teuk_ctx();
    if (c == nullptr) return fail(TEUK_ENOMEM, "host allocation failed");
    std::string err = teuk::build_geometry(d->M, d->a, d->s, d->m, d->nr, d->nth, d->rs_min, d->rs_max,
                                           d->cfl, d->rs_extract, c->G);
    if (err.empty()) err = ws_layout(c->G, row_pitch(c->G.nr), req, &c->lay);
    if (!err.empty()) {
        delete c;
        return fail(TEUK_EINVAL, err);
    }
    if (ws_bytes < c->lay.total) {
        const size_t need = c->lay.total;
        delete c;
        return fail(TEUK_ENOMEM, "workspace of " + std::to_string(ws_bytes) + " bytes, need " + std::to_string(need));
    }
    const Geometry& G = c->G;
    c->stream = static_cast<hipStream_t>(hip_stream);
    c->ws = static_cast<char*>(ws);
    c->ld = row_pitch(G.nr);
    c->ko_c = d->ko_eps / 16.0;
    c->nstrips = (G.nr + 61) / 62;
    {
        int dev = 0, cus = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
            c->nsimd = 4 * cus;
    }
    // default segment: 8 rows when that still gives at least one wave per
    // SIMD, else 4; the autotuner refines this by measurement.  The adjoint
    // runs 16-row segments where they give more waves than SIMDs (its
    // launches then run two waves per SIMD without source bodies and
    // without spills), else 4 (each wave alone on its SIMD: shorter
    // segments finish sooner).
    set_tuning_fields(c, (static_cast<long>(c->nstrips) * ((G.nth - 3) / 8 + 1) >= c->nsimd) ? 8 : 4, 1);
    set_adjoint_segment(c, (static_cast<long>(c->nstrips) * ((G.nth - 3) / 16 + 1) > c->nsimd) ? 16 : 4);
    const size_t plane_bytes = sizeof(double2) * static_cast<size_t>(c->ld) * G.nth;
    const WsLayout& L = c->lay;
    for (int l = 0; l < 2; ++l)
        for (int f = 0; f < 2; ++f)
            c->plane[l][f] = reinterpret_cast<double2*>(c->ws + L.planes + (2 * l + f) * plane_bytes);
    c->d_rnode = reinterpret_cast<double*>(c->ws + L.rnode);
    c->d_rhalf = reinterpret_cast<double*>(c->ws + L.rhalf);
    c->d_rows = reinterpret_cast<ThetaRow*>(c->ws + L.rows);
    c->d_flag = reinterpret_cast<int*>(c->ws + L.flag);
    if (L.win_r_cap > 0) {
        c->d_fh = reinterpret_cast<double2*>(c->ws + L.fh);
        c->d_fn = reinterpret_cast<double2*>(c->ws + L.fn);
        c->d_org = reinterpret_cast<int4*>(c->ws + L.org);
    }
    if (L.adjoint) {
        for (int l = 0; l < 2; ++l)
            for (int f = 0; f < 2; ++f)
                c->adj[l][f] = reinterpret_cast<double2*>(c->ws + L.adj + (2 * l + f) * plane_bytes);
        c->d_dA = reinterpret_cast<double*>(c->ws + L.dA);
        c->d_dA_part = reinterpret_cast<double*>(c->ws + L.dA_part);
        c->d_dA_blk = reinterpret_cast<double*>(c->ws + L.dA_blk);
    }
    const size_t rbytes = sizeof(double) * teuk::RF_COUNT * static_cast<size_t>(G.nr);
    hipError_t e = hipMemcpyAsync(c->d_rnode, G.rnode.data(), rbytes, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(c->d_rhalf, G.rhalf.data(), rbytes, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(c->d_rows, G.rows.data(), sizeof(ThetaRow) * G.nth, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = teuk::launch_zero(c->plane[0][0], 4 * plane_bytes, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        delete c;
        return hip_fail(e, "teuk_init_grid");
    }
    *out = c;
    return TEUK_OK;
}

extern "C" {

const char* teuk_last_error(void) { return g_last_error.c_str(); }

int teuk_workspace_size(const teuk_grid_desc* d, const teuk_ws_request* req, size_t* bytes) {
    if (d == nullptr || bytes == nullptr) return fail(TEUK_EINVAL, "null descriptor or output");
    *bytes = 0;
    if (!(d->ko_eps >= 0.0 && d->ko_eps <= 1.0)) return fail(TEUK_EINVAL, "need 0 <= ko_eps <= 1");
    teuk::Geometry G;
    std::string err = teuk::build_geometry(d->M, d->a, d->s, d->m, d->nr, d->nth, d->rs_min, d->rs_max, d->cfl,
                                           d->rs_extract, G);
    if (!err.empty()) return fail(TEUK_EINVAL, err);
    teuk_detail::WsLayout L;
    err = teuk_detail::ws_layout(G, row_pitch(G.nr), req, &L);
    if (!err.empty()) return fail(TEUK_EINVAL, err);
    *bytes = L.total;
    return TEUK_OK;
}

int teuk_init_grid(const teuk_grid_desc* d, const teuk_ws_request* req, void* hip_stream, void* ws,
                   size_t ws_bytes, teuk_ctx** out) {
    return teuk_detail::make_ctx(d, req, hip_stream, ws, ws_bytes, out);
}

int teuk_init_grid_static(const teuk_grid_desc* d, const teuk_ws_request* req, void* hip_stream, teuk_ctx** out) {
    if (d == nullptr || out == nullptr) return fail(TEUK_EINVAL, "null descriptor or output");
    *out = nullptr;
    size_t need = 0;
    if (int rc = teuk_workspace_size(d, req, &need)) return rc;
    if (need > teuk::kStaticWorkspaceBytes)
        return fail(TEUK_ENOMEM, "grid needs a workspace of " + std::to_string(need) +
                                     " bytes; the static workspace holds " +
                                     std::to_string(teuk::kStaticWorkspaceBytes));
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "static workspace device");
    void* ws = nullptr;
    HIP_TRY(teuk::static_workspace(&ws), "static workspace address");
    {
        std::lock_guard<std::mutex> lock(g_static_mutex);
        if (std::find(g_static_busy.begin(), g_static_busy.end(), dev) != g_static_busy.end())
            return fail(TEUK_ESTATE, "the static workspace of this device is held by another context");
        g_static_busy.push_back(dev);
    }
    const int rc = teuk_detail::make_ctx(d, req, hip_stream, ws, teuk::kStaticWorkspaceBytes, out);
    if (rc != TEUK_OK) {
        std::lock_guard<std::mutex> lock(g_static_mutex);
        g_static_busy.erase(std::remove(g_static_busy.begin(), g_static_busy.end(), dev), g_static_busy.end());
        return rc;
    }
    (*out)->static_dev = dev;
    return TEUK_OK;
}

int teuk_destroy(teuk_ctx* c) {
    if (c == nullptr) return TEUK_OK;
    if (c->in_batch) return fail(TEUK_EINVAL, "context belongs to a batch; destroy the batch");
    teuk_detail::destroy_ctx(c);
    return TEUK_OK;
}

int teuk_get_info(const teuk_ctx* c, teuk_info* out) {
    if (int rc = check_ctx(c)) return rc;
    if (out == nullptr) return fail(TEUK_EINVAL, "null output");
    out->dt = c->G.dt;
    out->h_r = c->G.h_r;
    out->h_th = c->G.h_th;
    out->r_plus = c->G.r_plus;
    out->r_minus = c->G.r_minus;
    out->i_ext = c->G.i_ext;
    out->nr = c->G.nr;
    out->nth = c->G.nth;
    out->row_pitch = c->ld;
    out->steps_done = c->steps_done;
    return TEUK_OK;
}

int teuk_set_state(teuk_ctx* c, const void* phi, const void* pi) {
    if (int rc = check_ctx(c)) return rc;
    if (phi == nullptr || pi == nullptr) return fail(TEUK_EINVAL, "null state pointer");
    const size_t w = sizeof(double2) * c->G.nr;
    HIP_TRY(hipMemcpy2DAsync(c->plane[c->cur][0], sizeof(double2) * c->ld, phi, w, w, c->G.nth,
                             hipMemcpyDeviceToDevice, c->stream), "set_state Phi");
    HIP_TRY(hipMemcpy2DAsync(c->plane[c->cur][1], sizeof(double2) * c->ld, pi, w, w, c->G.nth,
                             hipMemcpyDeviceToDevice, c->stream), "set_state Pi");
    c->steps_done = 0;
    c->batch_n0 = -1;
    c->batch_len = 0;
    return TEUK_OK;
}

int teuk_get_state(const teuk_ctx* c, void* phi, void* pi) {
    if (int rc = check_ctx(c)) return rc;
    if (phi == nullptr || pi == nullptr) return fail(TEUK_EINVAL, "null state pointer");
    const size_t w = sizeof(double2) * c->G.nr;
    HIP_TRY(hipMemcpy2DAsync(phi, w, c->plane[c->cur][0], sizeof(double2) * c->ld, w, c->G.nth,
                             hipMemcpyDeviceToDevice, c->stream), "get_state Phi");
    HIP_TRY(hipMemcpy2DAsync(pi, w, c->plane[c->cur][1], sizeof(double2) * c->ld, w, c->G.nth,
                             hipMemcpyDeviceToDevice, c->stream), "get_state Pi");
    return TEUK_OK;
}

int teuk_init_pulse(teuk_ctx* c, double center, double width, double amplitude) {
    if (int rc = check_ctx(c)) return rc;
    if (!(width > 0.0)) return fail(TEUK_EINVAL, "need width > 0");
    teuk::PulseParams Q;
    Q.phi = c->plane[c->cur][0];
    Q.pi = c->plane[c->cur][1];
    Q.ld = c->ld;
    Q.nr = c->G.nr;
    Q.nth = c->G.nth;
    Q.rpitch = c->G.nr;
    Q.rnode = c->d_rnode;
    Q.rnode_rs = c->d_rnode + static_cast<size_t>(teuk::RF_RS) * c->G.nr;
    Q.rows = c->d_rows;
    Q.center = center;
    Q.width = width;
    Q.amplitude = amplitude;
    Q.even = (std::abs(c->G.m) % 2 == 0);
    Q.kerr = (c->G.a != 0.0);
    HIP_TRY(teuk::launch_init_pulse(Q, c->stream), "init_pulse");
    c->steps_done = 0;
    c->batch_n0 = -1;
    c->batch_len = 0;
    return TEUK_OK;
}

int teuk_orbit_circular(double M, double a, double r0, double dt, int64_t nsamples, double* out) {
    if (out == nullptr || nsamples < 0) return fail(TEUK_EINVAL, "bad orbit output");
    if (!(M > 0.0) || !(std::fabs(a) < M)) return fail(TEUK_EINVAL, "need M > 0 and |a| < M");
    const double rp = M + std::sqrt(M * M - a * a);
    if (!(r0 > rp)) return fail(TEUK_EINVAL, "orbit radius inside the horizon");
    const double rsp = teuk::tortoise_of_x(r0 - rp, M, a);
    const double Om = std::sqrt(M) / (std::pow(r0, 1.5) + a * std::sqrt(M));
    for (int64_t k = 0; k < nsamples; ++k) {
        const double t = static_cast<double>(k) * (0.5 * dt);
        out[3 * k + 0] = rsp;
        out[3 * k + 1] = 0.5 * M_PI;
        out[3 * k + 2] = Om * t;
    }
    return TEUK_OK;
}

int teuk_set_source(teuk_ctx* c, const teuk_source_desc* s) {
    if (int rc = check_ctx(c)) return rc;
    HIP_TRY(hipStreamSynchronize(c->stream), "set_source sync");
    free_source(c);
    if (s == nullptr) return TEUK_OK;
    if (s->orbit == nullptr || s->nsamples < 2) return fail(TEUK_EINVAL, "orbit needs >= 2 samples");
    if (s->orbit_dev == nullptr) return fail(TEUK_EINVAL, "null orbit_dev (device buffer for the orbit)");
    if (!(s->sigma_r_cells > 0.0 && s->sigma_th_cells > 0.0 && s->cutoff_sigmas > 0.0))
        return fail(TEUK_EINVAL, "source widths and cutoff must be positive");
    const double wr = std::ceil(2.0 * s->cutoff_sigmas * s->sigma_r_cells) + 2.0;
    const double wt = std::ceil(2.0 * s->cutoff_sigmas * s->sigma_th_cells) + 2.0;
    if (!(wr <= c->lay.win_r_cap && wt <= c->lay.win_t_cap))
        return fail(TEUK_ENOMEM, "source footprint larger than the workspace was sized for (teuk_ws_request)");
    c->amplitude = s->amplitude;
    c->sig_r = s->sigma_r_cells * c->G.h_r;
    c->sig_th = s->sigma_th_cells * c->G.h_th;
    c->cut = s->cutoff_sigmas;
    c->win_r = static_cast<int>(wr);
    c->win_t = static_cast<int>(wt);
    c->nsamples = s->nsamples;
    const size_t obytes = sizeof(double) * 3 * static_cast<size_t>(s->nsamples);
    try {
        c->h_orbit.assign(s->orbit, s->orbit + 3 * static_cast<size_t>(s->nsamples));
    } catch (const std::bad_alloc&) {
        return fail(TEUK_ENOMEM, "host copy of the orbit");
    }
    hipError_t e = hipMemcpyAsync(s->orbit_dev, s->orbit, obytes, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        free_source(c);
        return hip_fail(e, "set_source");
    }
    c->d_orbit = static_cast<double*>(s->orbit_dev);
    c->has_src = true;
    return TEUK_OK;
}

int teuk_set_amplitude(teuk_ctx* c, double amplitude) {
    if (int rc = check_ctx(c)) return rc;
    if (!c->has_src) return fail(TEUK_ESTATE, "no source attached");
    c->amplitude = amplitude;
    return TEUK_OK;
}

int teuk_step_n(teuk_ctx* c, int64_t nsteps, void* waveform) {
    if (int rc = check_ctx(c)) return rc;
    if (nsteps < 0) return fail(TEUK_EINVAL, "negative step count");
    if (nsteps == 0) return TEUK_OK;
    const Geometry& G = c->G;
    if (c->has_src && 2 * (c->steps_done + nsteps - 1) + 1 >= c->nsamples)
        return fail(TEUK_ESTATE, "orbit has too few samples for the requested steps");
    teuk::StepParams P;
    P.rnode = c->d_rnode;
    P.rhalf = c->d_rhalf;
    P.rows = c->d_rows;
    P.nr = G.nr;
    P.nth = G.nth;
    P.ld = c->ld;
    P.rpitch = G.nr;
    P.nstrips = c->nstrips;
    P.nseg = c->nseg;
    P.dt = G.dt;
    P.inv_hr = 1.0 / G.h_r;
    P.ko_c = c->ko_c;
    P.even = (std::abs(G.m) % 2 == 0);
    P.kerr = (G.a != 0.0);
    P.i_ext = G.i_ext;
    P.win_r = c->win_r;
    P.win_t = c->win_t;
    P.frame_first = teuk::use_frame_first(c->nstrips * c->nseg, c->nsimd) ? 1 : 0;
    double2* wave = static_cast<double2*>(waveform);
    int64_t k = 0;
    while (k < nsteps) {
        const int64_t n = c->steps_done;
        // a blocked launch takes k_steps iterations; the remainder runs singly
        const int depth = (c->k_steps > 1 && nsteps - k >= c->k_steps) ? c->k_steps : 1;
        P.fh = P.fn = nullptr;
        P.org = nullptr;
        if (c->has_src) {
            size_t slot = 0;
            // a batch may run past this call, as far as the orbit has samples:
            // the last iteration it supports is (nsamples - 2) / 2 (needs sample 2n + 1)
            const int64_t span = (c->nsamples - 2) / 2 - n + 1;
            if (int rc = ensure_source(c, n, c->amplitude, false, span, &slot)) return rc;
            if (static_cast<int64_t>(slot) + depth > c->batch_len) {
                // the block's iterations must share one batch: start a new one at n
                // (an empty batch: any n would otherwise still count as resident)
                c->batch_n0 = -1;
                c->batch_len = 0;
                if (int rc = ensure_source(c, n, c->amplitude, false, span, &slot)) return rc;
            }
            const size_t wsz = static_cast<size_t>(c->win_r) * c->win_t;
            P.fh = c->d_fh + slot * wsz;
            P.fn = c->d_fn + slot * wsz;
            P.org = c->d_org + slot;
        }
        P.phi = c->plane[c->cur][0];
        P.pi = c->plane[c->cur][1];
        P.phi_out = c->plane[c->cur ^ 1][0];
        P.pi_out = c->plane[c->cur ^ 1][1];
        P.wave = wave ? wave + k * G.nth : nullptr;
        P.nstrips = (depth > 1) ? c->bstrips : c->nstrips;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (c->timing) {
            if (c->ev_used == kTimingPool)
                if (int rc = flush_timing(c)) return rc;
            while (c->ev_start.size() <= c->ev_used) {
                hipEvent_t a, b;
                HIP_TRY(hipEventCreate(&a), "event create");
                HIP_TRY(hipEventCreate(&b), "event create");
                c->ev_start.push_back(a);
                c->ev_stop.push_back(b);
            }
            e0 = c->ev_start[c->ev_used];
            e1 = c->ev_stop[c->ev_used];
            c->ev_used += 1;
        }
        if (depth > 1) {
            HIP_TRY(teuk::launch_block(P, c->seg_rows, depth, c->stream, e0, e1), "blocked step kernel");
        } else {
            HIP_TRY(teuk::launch_step(P, c->seg_rows, c->stream, e0, e1), "step kernel");
        }
        c->cur ^= 1;
        c->steps_done += depth;
        k += depth;
    }
    return TEUK_OK;
}

int teuk_adjoint_begin(teuk_ctx* c, const void* lam_phi, const void* lam_pi, int64_t n_end, const void* gw) {
    if (int rc = check_ctx(c)) return rc;
    if (n_end < 0) return fail(TEUK_EINVAL, "negative n_end");
    const Geometry& G = c->G;
    const size_t plane_bytes = sizeof(double2) * static_cast<size_t>(c->ld) * G.nth;
    if (!c->lay.adjoint)
        return fail(TEUK_ENOMEM, "the workspace has no adjoint area (teuk_ws_request.adjoint)");
    c->adj_cur = 0;
    double2* P0 = c->adj[0][0];
    double2* P1 = c->adj[0][1];
    const size_t w = sizeof(double2) * G.nr;
    if (lam_phi != nullptr) {
        HIP_TRY(hipMemcpy2DAsync(P0, sizeof(double2) * c->ld, lam_phi, w, w, G.nth, hipMemcpyDeviceToDevice,
                                 c->stream), "adjoint_begin copy");
    } else {
        HIP_TRY(teuk::launch_zero(P0, plane_bytes, c->stream), "adjoint_begin zero");
    }
    if (lam_pi != nullptr) {
        HIP_TRY(hipMemcpy2DAsync(P1, sizeof(double2) * c->ld, lam_pi, w, w, G.nth, hipMemcpyDeviceToDevice,
                                 c->stream), "adjoint_begin copy");
    } else {
        HIP_TRY(teuk::launch_zero(P1, plane_bytes, c->stream), "adjoint_begin zero");
    }
    if (gw != nullptr && n_end >= 1)
        HIP_TRY(teuk::launch_inject_column(P0, c->ld, G.nth, G.i_ext,
                                           static_cast<const double2*>(gw) + (n_end - 1) * G.nth, c->stream),
                "adjoint_begin inject");
    HIP_TRY(teuk::launch_zero(c->d_dA, sizeof(double), c->stream), "dA zero");
    c->part_filled = 0;
    c->adj_clock = n_end;
    return TEUK_OK;
}

int teuk_adjoint_step_n(teuk_ctx* c, int64_t nsteps, const void* gw) {
    if (int rc = check_ctx(c)) return rc;
    if (c->adj_clock < 0) return fail(TEUK_ESTATE, "teuk_adjoint_begin first");
    if (nsteps < 0 || nsteps > c->adj_clock) return fail(TEUK_EINVAL, "step count beyond iteration 0");
    const Geometry& G = c->G;
    if (c->has_src && 2 * (c->adj_clock - 1) + 1 >= c->nsamples && nsteps > 0)
        return fail(TEUK_ESTATE, "orbit has too few samples for the reverse sweep");
    teuk::AdjointParams P;
    P.rnode = c->d_rnode;
    P.rhalf = c->d_rhalf;
    P.rows = c->d_rows;
    P.nr = G.nr;
    P.nth = G.nth;
    P.ld = c->ld;
    P.nstrips = c->nstrips;
    P.nseg = c->adj_nseg;
    P.dt = G.dt;
    P.inv_hr = 1.0 / G.h_r;
    P.ko_c = c->ko_c;
    P.even = (std::abs(G.m) % 2 == 0);
    P.kerr = (G.a != 0.0);
    P.i_ext = G.i_ext;
    P.win_r = c->win_r;
    P.win_t = c->win_t;
    P.sub_s0 = P.sub_ns = P.sub_g0 = P.sub_ng = 0;
    const int items = c->nstrips * c->adj_nseg;
    P.frame_first = teuk::use_frame_first(items, c->nsimd) ? 1 : 0;
    if (c->part_items != items) {
        if (int rc = flush_partials(c)) return rc;
        c->part_items = items;
    }
    bool by_window = false;
    for (int64_t k = 0; k < nsteps; ++k) {
        const int64_t m = c->adj_clock - 1;
        P.fh = P.fn = nullptr;
        P.org = nullptr;
        P.dA_part = nullptr;
        if (c->has_src) {
            size_t slot = 0;
            if (int rc = ensure_source(c, m, 1.0, true, m + 1, &slot)) return rc;
            const size_t wsz = static_cast<size_t>(c->win_r) * c->win_t;
            P.fh = c->d_fh + slot * wsz;
            P.fn = c->d_fn + slot * wsz;
            P.org = c->d_org + slot;
            by_window = false;
            if (teuk::adjoint_rect_fits(c->nstrips, c->adj_nseg)) {
                int s0, ns, g0, ng, r_lo, r_hi;
                source_items(c, m, c->adj_seg_rows, c->adj_nseg, s0, ns, g0, ng, r_lo, r_hi);
                P.sub_s0 = static_cast<int16_t>(s0);
                P.sub_ns = static_cast<int16_t>(ns);
                P.sub_g0 = static_cast<int16_t>(g0);
                P.sub_ng = static_cast<int16_t>(ng);
                // rows [r_lo, r_hi) hold both windows with a 2-row margin
                by_window = r_lo >= 3 && r_hi <= G.nth - 3;
            }
            if (c->part_filled == kPartSteps)
                if (int rc = flush_partials(c)) return rc;
            P.dA_part = c->d_dA_part + static_cast<size_t>(c->part_filled) * items;
            c->part_filled += 1;
        }
        P.gw = (gw != nullptr && m >= 1) ? static_cast<const double2*>(gw) + (m - 1) * G.nth : nullptr;
        P.lam_phi = c->adj[c->adj_cur][0];
        P.lam_pi = c->adj[c->adj_cur][1];
        P.out_phi = c->adj[c->adj_cur ^ 1][0];
        P.out_pi = c->adj[c->adj_cur ^ 1][1];
        HIP_TRY(teuk::launch_adjoint(P, c->adj_seg_rows, c->nsimd, c->stream, by_window), "adjoint kernel");
        c->adj_cur ^= 1;
        c->adj_clock = m;
    }
    return TEUK_OK;
}

int teuk_adjoint_add_state(teuk_ctx* c, const void* gphi, const void* gpi) {
    if (int rc = check_ctx(c)) return rc;
    if (c->adj_clock < 0) return fail(TEUK_ESTATE, "teuk_adjoint_begin first");
    HIP_TRY(teuk::launch_add_planes(c->adj[c->adj_cur][0], c->adj[c->adj_cur][1],
                                    static_cast<const double2*>(gphi), static_cast<const double2*>(gpi),
                                    c->G.nr, c->G.nth, c->ld, c->stream), "adjoint_add_state");
    return TEUK_OK;
}

int teuk_adjoint_get(teuk_ctx* c, void* lam_phi, void* lam_pi, double* dL_dA) {
    if (int rc = check_ctx(c)) return rc;
    if (c->adj_clock < 0) return fail(TEUK_ESTATE, "teuk_adjoint_begin first");
    const size_t w = sizeof(double2) * c->G.nr;
    if (lam_phi != nullptr)
        HIP_TRY(hipMemcpy2DAsync(lam_phi, w, c->adj[c->adj_cur][0], sizeof(double2) * c->ld, w, c->G.nth,
                                 hipMemcpyDeviceToDevice, c->stream), "adjoint_get");
    if (lam_pi != nullptr)
        HIP_TRY(hipMemcpy2DAsync(lam_pi, w, c->adj[c->adj_cur][1], sizeof(double2) * c->ld, w, c->G.nth,
                                 hipMemcpyDeviceToDevice, c->stream), "adjoint_get");
    if (dL_dA != nullptr) {
        if (int rc = flush_partials(c)) return rc;
        HIP_TRY(hipMemcpyAsync(dL_dA, c->d_dA, sizeof(double), hipMemcpyDeviceToHost, c->stream), "dA copy");
        HIP_TRY(hipStreamSynchronize(c->stream), "adjoint_get sync");
    }
    return TEUK_OK;
}

static int check_plan(const teuk_ctx* c, const teuk_grad_plan* p, int64_t* interval) {
    if (p == nullptr) return fail(TEUK_EINVAL, "null plan");
    if (p->nsteps < 1) return fail(TEUK_EINVAL, "plan needs nsteps >= 1");
    if (p->snapshots < 0) return fail(TEUK_EINVAL, "snapshots must be >= 0");
    if (p->snapshots > 0 && p->interval != 0)
        return fail(TEUK_EINVAL, "a binomial plan (snapshots > 0) takes interval 0");
    int64_t iv = p->interval;
    if (iv == 0) iv = static_cast<int64_t>(std::ceil(std::sqrt(static_cast<double>(p->nsteps))));
    if (iv < 1) return fail(TEUK_EINVAL, "interval must be >= 0");
    if (p->state_weight != 0.0) {
        if (!(0 <= p->i0 && p->i0 < p->i1 && p->i1 <= c->G.nr && 0 <= p->j0 && p->j0 < p->j1 &&
              p->j1 <= c->G.nth))
            return fail(TEUK_EINVAL, "loss rectangle outside the grid");
        if (!(1 <= p->n_lo && p->n_lo <= p->n_hi && p->n_hi <= p->nsteps))
            return fail(TEUK_EINVAL, "need 1 <= n_lo <= n_hi <= nsteps");
    }
    *interval = iv;
    return TEUK_OK;
}

}  // extern "C"

namespace {

// Byte offsets inside a plan's checkpoint buffer: 2K snapshot planes (K =
// the uniform schedule's snapshot count, or the binomial schedule's slots),
// then (state loss only) the rectangle buffer (uniform schedule only), the
// loss sum and its partials.
struct CkptLayout {
    size_t snaps = 0, seg = 0, ls = 0, ls_part = 0, total = 0;
};

CkptLayout ckpt_layout(const teuk_ctx* c, const teuk_grad_plan* p, int64_t iv) {
    CkptLayout L;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t at = off;
        off += (bytes + 255) / 256 * 256;
        return at;
    };
    const size_t plane_bytes = sizeof(double2) * static_cast<size_t>(c->ld) * c->G.nth;
    const bool binomial = p->snapshots > 0;
    const int64_t K = binomial ? p->snapshots : (p->nsteps + iv - 1) / iv;
    L.snaps = take(2 * static_cast<size_t>(K) * plane_bytes);
    if (p->state_weight != 0.0) {
        const size_t wr = static_cast<size_t>(p->i1 - p->i0), hr = static_cast<size_t>(p->j1 - p->j0);
        L.seg = take(binomial ? 0 : sizeof(double2) * wr * hr * static_cast<size_t>(iv));
        L.ls = take(sizeof(double));
        L.ls_part = take(sizeof(double) * (c->G.nth + teuk::reduce_partials_blocks(c->G.nth)));
    }
    L.total = off;
    return L;
}

// Point the context's checkpoint buffers into the plan's caller-owned buffer.
int bind_ckpt(teuk_ctx* c, const teuk_grad_plan* p, int64_t iv) {
    if (!c->lay.adjoint)
        return fail(TEUK_ENOMEM, "the workspace has no adjoint area (teuk_ws_request.adjoint)");
    const CkptLayout L = ckpt_layout(c, p, iv);
    if (p->ckpt_dev == nullptr) return fail(TEUK_EINVAL, "null checkpoint buffer (plan.ckpt_dev)");
    if (reinterpret_cast<uintptr_t>(p->ckpt_dev) % 256 != 0)
        return fail(TEUK_EINVAL, "checkpoint buffer must be 256-byte aligned");
    if (p->ckpt_bytes < L.total)
        return fail(TEUK_ENOMEM, "checkpoint buffer of " + std::to_string(p->ckpt_bytes) + " bytes, need " +
                                     std::to_string(L.total));
    char* base = static_cast<char*>(p->ckpt_dev);
    c->snaps = reinterpret_cast<double2*>(base + L.snaps);
    const bool sl = p->state_weight != 0.0;
    c->seg_buf = (sl && p->snapshots == 0) ? reinterpret_cast<double2*>(base + L.seg) : nullptr;
    c->d_ls = sl ? reinterpret_cast<double*>(base + L.ls) : nullptr;
    c->d_ls_part = sl ? reinterpret_cast<double*>(base + L.ls_part) : nullptr;
    return TEUK_OK;
}

}  // namespace

extern "C" {

int teuk_checkpoint_schedule(int64_t nsteps, int64_t snapshots, int32_t phase, int64_t* actions, int64_t cap,
                             int64_t* count, int64_t* stats) {
    if (count == nullptr) return fail(TEUK_EINVAL, "null count");
    *count = 0;
    if (nsteps < 1 || snapshots < 1) return fail(TEUK_EINVAL, "need nsteps >= 1 and snapshots >= 1");
    if (phase != 0 && phase != 1) return fail(TEUK_EINVAL, "phase must be 0 (forward) or 1 (backward)");
    if (cap < 0 || (cap > 0 && actions == nullptr)) return fail(TEUK_EINVAL, "bad action buffer");
    teuk_detail::RevolveSchedule S;
    if (!teuk_detail::revolve_schedule(nsteps, snapshots, &S)) return fail(TEUK_EINVAL, "no schedule");
    const auto& list = phase == 0 ? S.forward : S.backward;
    *count = static_cast<int64_t>(list.size());
    const int64_t n = std::min<int64_t>(cap, *count);
    for (int64_t k = 0; k < n; ++k) {
        actions[3 * k] = list[k].op;
        actions[3 * k + 1] = list[k].a;
        actions[3 * k + 2] = list[k].b;
    }
    if (stats != nullptr) {
        stats[0] = S.repetitions;
        stats[1] = S.backward_advances;
        stats[2] = S.slots_used;
    }
    return TEUK_OK;
}

namespace {

// Copy the current state into snapshot slot k, or back.
int snapshot_copy(teuk_ctx* c, int64_t k, bool restore) {
    const size_t plane_bytes = sizeof(double2) * static_cast<size_t>(c->ld) * c->G.nth;
    const size_t plane_elems = plane_bytes / sizeof(double2);
    for (int f = 0; f < 2; ++f) {
        double2* snap = c->snaps + (2 * k + f) * plane_elems;
        double2* cur = c->plane[c->cur][f];
        HIP_TRY(hipMemcpyAsync(restore ? cur : snap, restore ? snap : cur, plane_bytes, hipMemcpyDeviceToDevice,
                               c->stream), restore ? "restore" : "snapshot");
    }
    return TEUK_OK;
}

// Add |Phi^n|^2 on the plan's rectangle to the loss sum (phi: the Phi plane
// holding u^n).
int accumulate_state_loss(teuk_ctx* c, const teuk_grad_plan* p, const double2* phi) {
    HIP_TRY(teuk::launch_region_sumsq(phi, c->ld, p->i0, p->i1, p->j0, p->j1, c->d_ls_part, c->stream),
            "state loss");
    HIP_TRY(teuk::launch_reduce_partials(c->d_ls_part, p->j1 - p->j0, c->d_ls_part + c->G.nth, c->d_ls,
                                         c->stream), "state loss reduction");
    return TEUK_OK;
}

// Runs the actions of a binomial schedule.  The current state may live in a
// snapshot slot: a restore only names the slot, the next iteration reads its
// input from there, and the iteration that precedes a store writes its
// output straight into the slot, so no state is copied except the caller's
// u^0 (and, at the end, the last state back into the context's level).
struct RevolveRunner {
    teuk_ctx* c;
    const teuk_grad_plan* p;
    size_t plane_elems;
    int64_t src = -1;   // slot holding the current state; -1: the context's current level

    double2* slot_plane(int64_t k, int f) const { return c->snaps + (2 * k + f) * plane_elems; }
    double2* cur_phi() const { return src >= 0 ? slot_plane(src, 0) : c->plane[c->cur][0]; }

    // One iteration from the current state, its output into slot to_slot
    // (-1: the context's other level).
    int step_once(int64_t to_slot, double2* wave) {
        double2* saved[2][2];
        std::memcpy(saved, c->plane, sizeof(saved));
        const int r = c->cur, w = c->cur ^ 1;
        for (int f = 0; f < 2; ++f) {
            if (src >= 0) c->plane[r][f] = slot_plane(src, f);
            if (to_slot >= 0) c->plane[w][f] = slot_plane(to_slot, f);
        }
        const int rc = teuk_step_n(c, 1, wave);
        std::memcpy(c->plane, saved, sizeof(saved));
        if (rc) return rc;
        src = to_slot;
        return TEUK_OK;
    }

    // k iterations; store_slot >= 0: the last one writes into that slot.
    // with_loss: accumulate the state loss over the plan's window.
    int advance(int64_t k, int64_t store_slot, double2* wave, bool with_loss) {
        const int nth = c->G.nth;
        int64_t done = 0;
        while (done < k) {
            const int64_t n = c->steps_done;
            const bool last = done == k - 1;
            const bool in_win = with_loss && n + 1 >= p->n_lo && n + 1 <= p->n_hi;
            if (src >= 0 || (last && store_slot >= 0) || in_win) {
                if (int rc = step_once(last ? store_slot : -1, wave ? wave + n * nth : nullptr)) return rc;
                done += 1;
                if (in_win)
                    if (int rc = accumulate_state_loss(c, p, cur_phi())) return rc;
                continue;
            }
            int64_t run = k - done - (store_slot >= 0 ? 1 : 0);
            if (with_loss && n + 1 < p->n_lo) run = std::min(run, p->n_lo - 1 - n);
            if (int rc = teuk_step_n(c, run, wave ? wave + n * nth : nullptr)) return rc;
            done += run;
        }
        return TEUK_OK;
    }

    // Copy the current state into slot k (only the caller's u^0 needs this).
    int store_copy(int64_t k) {
        const size_t plane_bytes = plane_elems * sizeof(double2);
        for (int f = 0; f < 2; ++f) {
            const double2* from = src >= 0 ? slot_plane(src, f) : c->plane[c->cur][f];
            HIP_TRY(hipMemcpyAsync(slot_plane(k, f), from, plane_bytes, hipMemcpyDeviceToDevice, c->stream),
                    "snapshot");
        }
        src = k;
        return TEUK_OK;
    }

    // Leave the current state in the context's level.
    int materialize() {
        if (src < 0) return TEUK_OK;
        const size_t plane_bytes = plane_elems * sizeof(double2);
        for (int f = 0; f < 2; ++f)
            HIP_TRY(hipMemcpyAsync(c->plane[c->cur][f], slot_plane(src, f), plane_bytes, hipMemcpyDeviceToDevice,
                                   c->stream), "restore");
        src = -1;
        return TEUK_OK;
    }

    int run(const std::vector<teuk_detail::RevolveAction>& acts, double2* wave, bool with_loss, const void* gw,
            double scale) {
        const bool sl = p->state_weight != 0.0;
        for (size_t i = 0; i < acts.size(); ++i) {
            const auto& act = acts[i];
            switch (act.op) {
                case teuk_detail::kAdvance: {
                    // a store right after an advance takes the advance's last output
                    const bool then_store = i + 1 < acts.size() && acts[i + 1].op == teuk_detail::kStore;
                    if (int rc = advance(act.a, then_store ? acts[i + 1].a : -1, wave, with_loss)) return rc;
                    if (then_store) ++i;
                    break;
                }
                case teuk_detail::kStore:
                    if (int rc = store_copy(act.a)) return rc;
                    break;
                case teuk_detail::kRestore:
                    src = act.a;
                    c->steps_done = act.b;
                    break;
                default: {
                    const int64_t m = act.a;
                    if (c->steps_done != m || c->adj_clock != m + 1)
                        return fail(TEUK_ESTATE, "checkpoint schedule out of order");
                    if (int rc = teuk_adjoint_step_n(c, 1, gw)) return rc;
                    if (sl && m >= 1 && m >= p->n_lo && m <= p->n_hi)
                        HIP_TRY(teuk::launch_add_region(c->adj[c->adj_cur][0], c->ld, cur_phi(), c->ld, false,
                                                        scale, p->i0, p->i1, p->j0, p->j1, c->stream),
                                "state grad");
                }
            }
        }
        return materialize();
    }
};

// Forward of a binomial plan: the schedule's stores on the way to u^nsteps.
int forward_binomial(teuk_ctx* c, const teuk_grad_plan* p, double2* wave) {
    teuk_detail::RevolveSchedule S;
    if (!teuk_detail::revolve_schedule(p->nsteps, p->snapshots, &S)) return fail(TEUK_EINVAL, "no schedule");
    RevolveRunner R{c, p, static_cast<size_t>(c->ld) * c->G.nth};
    return R.run(S.forward, wave, p->state_weight != 0.0, nullptr, 0.0);
}

// Backward of a binomial plan from u^nsteps: restores, recomputes and
// reverse iterations in the schedule's order.
int backward_binomial(teuk_ctx* c, const teuk_grad_plan* p, const void* gw, double scale) {
    teuk_detail::RevolveSchedule S;
    if (!teuk_detail::revolve_schedule(p->nsteps, p->snapshots, &S)) return fail(TEUK_EINVAL, "no schedule");
    RevolveRunner R{c, p, static_cast<size_t>(c->ld) * c->G.nth};
    return R.run(S.backward, nullptr, false, gw, scale);
}

}  // namespace

int teuk_checkpoint_size(const teuk_ctx* c, const teuk_grad_plan* plan, size_t* bytes) {
    if (int rc = check_ctx(c)) return rc;
    if (bytes == nullptr) return fail(TEUK_EINVAL, "null output");
    *bytes = 0;
    int64_t iv = 0;
    if (int rc = check_plan(c, plan, &iv)) return rc;
    *bytes = ckpt_layout(c, plan, iv).total;
    return TEUK_OK;
}

int teuk_forward_checkpointed(teuk_ctx* c, const teuk_grad_plan* plan, void* waveform, double* state_loss) {
    if (int rc = check_ctx(c)) return rc;
    int64_t iv = 0;
    if (int rc = check_plan(c, plan, &iv)) return rc;
    if (c->steps_done != 0) return fail(TEUK_ESTATE, "set the initial state first (no iteration taken since)");
    c->ckpt_valid = false;
    if (int rc = bind_ckpt(c, plan, iv)) return rc;
    const Geometry& G = c->G;
    const int64_t N = plan->nsteps;
    const bool sl = plan->state_weight != 0.0;
    if (sl) HIP_TRY(teuk::launch_zero(c->d_ls, sizeof(double), c->stream), "state loss zero");
    double2* wave = static_cast<double2*>(waveform);
    if (plan->snapshots > 0) {
        if (int rc = forward_binomial(c, plan, wave)) return rc;
    } else {
        const int64_t K = (N + iv - 1) / iv;
        for (int64_t k = 0; k < K; ++k) {
            const int64_t s0 = k * iv, s1 = std::min(s0 + iv, N);
            if (int rc = snapshot_copy(c, k, false)) return rc;
            const bool touches = sl && !(s1 < plan->n_lo || s0 + 1 > plan->n_hi);
            if (!touches) {
                if (int rc = teuk_step_n(c, s1 - s0, wave ? wave + s0 * G.nth : nullptr)) return rc;
                continue;
            }
            for (int64_t n = s0; n < s1; ++n) {
                if (int rc = teuk_step_n(c, 1, wave ? wave + n * G.nth : nullptr)) return rc;
                if (n + 1 >= plan->n_lo && n + 1 <= plan->n_hi)
                    if (int rc = accumulate_state_loss(c, plan, c->plane[c->cur][0])) return rc;
            }
        }
    }
    if (state_loss != nullptr) {
        double acc = 0.0;
        if (sl) {
            HIP_TRY(hipMemcpyAsync(&acc, c->d_ls, sizeof(double), hipMemcpyDeviceToHost, c->stream), "loss copy");
            HIP_TRY(hipStreamSynchronize(c->stream), "loss sync");
        }
        *state_loss = plan->state_weight * acc;
    }
    c->ckpt_plan = *plan;
    c->ckpt_valid = true;
    return TEUK_OK;
}

int teuk_backward_checkpointed(teuk_ctx* c, const teuk_grad_plan* plan, const void* gw, double dL_dLs,
                               void* grad_phi0, void* grad_pi0, double* dL_dA) {
    if (int rc = check_ctx(c)) return rc;
    int64_t iv = 0;
    if (int rc = check_plan(c, plan, &iv)) return rc;
    if (!c->ckpt_valid || std::memcmp(&c->ckpt_plan, plan, sizeof(teuk_grad_plan)) != 0 ||
        c->steps_done != plan->nsteps)
        return fail(TEUK_ESTATE, "run teuk_forward_checkpointed with the same plan first");
    const int64_t N = plan->nsteps;
    const bool sl = plan->state_weight != 0.0;
    const bool recompute = sl || plan->force_recompute != 0;
    const double scale = 2.0 * plan->state_weight * dL_dLs;
    const int wr = plan->i1 - plan->i0, hr = plan->j1 - plan->j0;
    if (int rc = teuk_adjoint_begin(c, nullptr, nullptr, N, gw)) return rc;
    if (sl && N >= plan->n_lo && N <= plan->n_hi)
        HIP_TRY(teuk::launch_add_region(c->adj[c->adj_cur][0], c->ld, c->plane[c->cur][0], c->ld, false, scale,
                                        plan->i0, plan->i1, plan->j0, plan->j1, c->stream), "state grad");
    if (!recompute) {
        // the reverse sweep needs no forward state
        if (int rc = teuk_adjoint_step_n(c, N, gw)) return rc;
    } else if (plan->snapshots > 0) {
        if (int rc = backward_binomial(c, plan, gw, scale)) return rc;
    } else {
        const int64_t K = (N + iv - 1) / iv;
        for (int64_t k = K - 1; k >= 0; --k) {
            const int64_t s0 = k * iv, s1 = std::min(s0 + iv, N);
            // restore u^{s0} and recompute the segment, keeping Phi on the rectangle
            if (int rc = snapshot_copy(c, k, true)) return rc;
            c->steps_done = s0;
            for (int64_t m = s0; m < s1; ++m) {
                if (sl && m >= plan->n_lo && m <= plan->n_hi)
                    HIP_TRY(hipMemcpy2DAsync(c->seg_buf + static_cast<size_t>(m - s0) * wr * hr,
                                             sizeof(double2) * wr,
                                             c->plane[c->cur][0] + static_cast<size_t>(plan->j0) * c->ld + plan->i0,
                                             sizeof(double2) * c->ld, sizeof(double2) * wr, hr,
                                             hipMemcpyDeviceToDevice, c->stream), "segment store");
                if (m + 1 < s1)
                    if (int rc = teuk_step_n(c, 1, nullptr)) return rc;
            }
            for (int64_t m = s1 - 1; m >= s0; --m) {
                if (int rc = teuk_adjoint_step_n(c, 1, gw)) return rc;
                if (sl && m >= 1 && m >= plan->n_lo && m <= plan->n_hi)
                    HIP_TRY(teuk::launch_add_region(c->adj[c->adj_cur][0], c->ld,
                                                    c->seg_buf + static_cast<size_t>(m - s0) * wr * hr, wr, true,
                                                    scale, plan->i0, plan->i1, plan->j0, plan->j1, c->stream),
                            "state grad");
            }
        }
    }
    c->ckpt_valid = false;
    return teuk_adjoint_get(c, grad_phi0, grad_pi0, dL_dA);
}

int teuk_extract_waveform(const teuk_ctx* c, void* out) {
    if (int rc = check_ctx(c)) return rc;
    if (out == nullptr) return fail(TEUK_EINVAL, "null output");
    HIP_TRY(hipMemcpy2DAsync(out, sizeof(double2), c->plane[c->cur][0] + c->G.i_ext,
                             sizeof(double2) * c->ld, sizeof(double2), c->G.nth, hipMemcpyDeviceToDevice,
                             c->stream), "extract");
    return TEUK_OK;
}

int teuk_set_tuning(teuk_ctx* c, const teuk_tuning* t) {
    if (int rc = check_ctx(c)) return rc;
    if (t == nullptr) return fail(TEUK_EINVAL, "null tuning");
    if (t->k_steps == 1) {
        if (!teuk::valid_segment_rows(t->seg_rows)) return fail(TEUK_EINVAL, "seg_rows must be 4, 8 or 16");
    } else if (!teuk::valid_block(t->seg_rows, t->k_steps)) {
        return fail(TEUK_EINVAL, "no blocked variant for this (seg_rows, k_steps); valid: (4,2), (8,2), (4,4)");
    }
    if (t->adj_seg_rows != 0 && !teuk::valid_segment_rows(t->adj_seg_rows))
        return fail(TEUK_EINVAL, "adj_seg_rows must be 0, 4, 8 or 16");
    set_tuning_fields(c, t->seg_rows, t->k_steps);
    if (t->adj_seg_rows != 0) set_adjoint_segment(c, t->adj_seg_rows);
    return TEUK_OK;
}

int teuk_get_tuning(const teuk_ctx* c, teuk_tuning* out) {
    if (int rc = check_ctx(c)) return rc;
    if (out == nullptr) return fail(TEUK_EINVAL, "null output");
    out->seg_rows = c->seg_rows;
    out->k_steps = c->k_steps;
    out->adj_seg_rows = c->adj_seg_rows;
    return TEUK_OK;
}

int teuk_autotune(teuk_ctx* c, const char* cache_path, teuk_tune_entry* table, int32_t capacity,
                  int32_t* count) {
    if (int rc = check_ctx(c)) return rc;
    if (count != nullptr) *count = 0;
    if (table != nullptr && capacity < 0) return fail(TEUK_EINVAL, "negative table capacity");
    const Geometry& G = c->G;
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev), "autotune device");
    hipDeviceProp_t prop;
    HIP_TRY(hipGetDeviceProperties(&prop, dev), "autotune device properties");
    std::string arch = prop.gcnArchName;
    arch = arch.substr(0, arch.find(':'));
    // Trials: kWarm untimed then kReps timed runs of kIters iterations per
    // candidate, one after another from the current iteration.  They run
    // with the context's source when its orbit table covers them all (the
    // waves that meet a window take the longer general body, and how long
    // they make a launch depends on the segment length), else without.
    constexpr int kWarm = 8, kIters = 32, kReps = 3;   // multiples of every blocked depth
    constexpr int kCandidates = sizeof(teuk::kSegVariants) / sizeof(teuk::kSegVariants[0]) +
                                sizeof(teuk::kBlockVariants) / sizeof(teuk::kBlockVariants[0]);
    const int64_t trial_iters = static_cast<int64_t>(kCandidates) * (kWarm + kReps * kIters);
    const bool with_src = c->has_src && 2 * (c->steps_done + trial_iters) + 1 < c->nsamples;
    char keybuf[256];
    std::snprintf(keybuf, sizeof(keybuf), "%s nr=%d nth=%d kerr=%d ko=%d source=%d src=%s", arch.c_str(), G.nr,
                  G.nth, G.a != 0.0 ? 1 : 0, c->ko_c != 0.0 ? 1 : 0, with_src ? 1 : 0, TEUK_SOURCE_HASH);
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
        bool found = false;
        teuk_tune_entry hit{};
        std::string line;
        while (f && std::getline(f, line)) {
            std::istringstream ls(line);
            std::string k, seg, kk, us;
            if (!std::getline(ls, k, '\t') || !std::getline(ls, seg, '\t') || !std::getline(ls, kk, '\t') ||
                !std::getline(ls, us, '\t'))
                continue;
            if (k != key) continue;
            teuk_tune_entry e{};
            e.seg_rows = std::atoi(seg.c_str());
            e.k_steps = std::atoi(kk.c_str());
            e.us_per_iteration = std::atof(us.c_str());
            const bool ok = (e.k_steps == 1) ? teuk::valid_segment_rows(e.seg_rows)
                                             : teuk::valid_block(e.seg_rows, e.k_steps);
            if (ok) {
                hit = e;
                found = true;
            }
        }
        if (found) {
            set_tuning_fields(c, hit.seg_rows, hit.k_steps);
            emit({hit});
            return TEUK_OK;
        }
    }

    std::vector<teuk_tune_entry> cand;
    for (int seg : teuk::kSegVariants) cand.push_back({seg, 1, 0, 0.0});
    for (const auto& v : teuk::kBlockVariants) cand.push_back({v.seg, v.k, 0, 0.0});

    // save what the trials disturb
    const size_t plane_bytes = sizeof(double2) * static_cast<size_t>(c->ld) * G.nth;
    const int cur0 = c->cur;
    const int64_t steps0 = c->steps_done;
    const bool src0 = c->has_src;
    const bool timing0 = c->timing;
    const int seg0 = c->seg_rows, k0 = c->k_steps;
    hipEvent_t ev[2] = {nullptr, nullptr};
    if (int rc = flush_timing(c)) return rc;
    // the current level goes to host memory for the trials
    std::vector<double2> save[2];
    try {
        for (auto& v : save) v.resize(plane_bytes / sizeof(double2));
    } catch (const std::bad_alloc&) {
        return fail(TEUK_ENOMEM, "autotune: host copy of the state");
    }
    HIP_TRY(hipStreamSynchronize(c->stream), "autotune sync");
    for (int f = 0; f < 2; ++f)
        HIP_TRY(hipMemcpy(save[f].data(), c->plane[cur0][f], plane_bytes, hipMemcpyDeviceToHost), "autotune save");
    auto restore = [&]() {
        (void)hipStreamSynchronize(c->stream);
        c->cur = cur0;
        for (int f = 0; f < 2; ++f)
            (void)hipMemcpy(c->plane[cur0][f], save[f].data(), plane_bytes, hipMemcpyHostToDevice);
        c->steps_done = steps0;
        c->has_src = src0;
        c->timing = timing0;
        for (auto& x : ev)
            if (x != nullptr) (void)hipEventDestroy(x);
    };
    hipError_t e = hipEventCreate(&ev[0]);
    if (e == hipSuccess) e = hipEventCreate(&ev[1]);
    if (e != hipSuccess) {
        restore();
        set_tuning_fields(c, seg0, k0);
        return hip_fail(e, "autotune setup");
    }
    c->has_src = with_src;
    c->timing = false;
    for (auto& t : cand) {
        set_tuning_fields(c, t.seg_rows, t.k_steps);
        int rc = teuk_step_n(c, kWarm, nullptr);
        double best = 1e300;
        for (int r = 0; rc == TEUK_OK && r < kReps; ++r) {
            float ms = 0.0f;
            e = hipEventRecord(ev[0], c->stream);
            if (e == hipSuccess) rc = teuk_step_n(c, kIters, nullptr);
            if (e == hipSuccess && rc == TEUK_OK) e = hipEventRecord(ev[1], c->stream);
            if (e == hipSuccess && rc == TEUK_OK) e = hipEventSynchronize(ev[1]);
            if (e == hipSuccess && rc == TEUK_OK) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
            if (e != hipSuccess && rc == TEUK_OK) rc = hip_fail(e, "autotune timing");
            best = std::min(best, 1e3 * static_cast<double>(ms) / kIters);
        }
        if (rc != TEUK_OK) {
            const std::string msg = g_last_error;
            restore();
            set_tuning_fields(c, seg0, k0);
            return fail(rc, msg);
        }
        t.us_per_iteration = best;
    }
    restore();
    std::stable_sort(cand.begin(), cand.end(), [](const teuk_tune_entry& a, const teuk_tune_entry& b) {
        return a.us_per_iteration < b.us_per_iteration;
    });
    set_tuning_fields(c, cand[0].seg_rows, cand[0].k_steps);
    emit(cand);
    if (cache_path != nullptr) {
        std::ofstream f(cache_path, std::ios::app);
        char line[512];
        std::snprintf(line, sizeof(line), "%s\t%d\t%d\t%.4f\n", key.c_str(), cand[0].seg_rows, cand[0].k_steps,
                      cand[0].us_per_iteration);
        if (!(f << line)) return fail(TEUK_EINVAL, std::string("cannot append to tuning cache ") + cache_path);
    }
    return TEUK_OK;
}

static int check_flux(const teuk_flux_desc* d, size_t* h_bytes) {
    if (d == nullptr) return fail(TEUK_EINVAL, "null flux descriptor");
    if (d->nmodes < 1 || d->nmodes > teuk::kMaxFluxModes) return fail(TEUK_EINVAL, "need 1 <= nmodes <= 16");
    if (d->m == nullptr || d->waves == nullptr) return fail(TEUK_EINVAL, "null m or waves array");
    if (d->nsteps < 0 || d->nth < 3) return fail(TEUK_EINVAL, "need nsteps >= 0 and nth >= 3");
    if (!(d->dt > 0.0)) return fail(TEUK_EINVAL, "need dt > 0");
    for (int k = 0; k < d->nmodes; ++k) {
        if (d->waves[k] == nullptr) return fail(TEUK_EINVAL, "null waveform " + std::to_string(k));
        for (int l = 0; l < k; ++l)
            if (d->m[l] == d->m[k]) return fail(TEUK_EINVAL, "the m of the waveforms must be distinct");
    }
    const size_t rows = static_cast<size_t>(d->nsteps) + 1;
    *h_bytes = (sizeof(double2) * d->nmodes * rows * d->nth + 255) / 256 * 256;
    return TEUK_OK;
}

int teuk_flux_workspace_size(const teuk_flux_desc* d, size_t* bytes) {
    if (bytes == nullptr) return fail(TEUK_EINVAL, "null output");
    *bytes = 0;
    size_t hb = 0;
    if (int rc = check_flux(d, &hb)) return rc;
    *bytes = 2 * hb;     // H, then K
    return TEUK_OK;
}

int teuk_radiated_flux(const teuk_flux_desc* d, void* hip_stream, void* ws, size_t ws_bytes, void* out) {
    size_t hb = 0;
    if (int rc = check_flux(d, &hb)) return rc;
    if (out == nullptr) return fail(TEUK_EINVAL, "null output");
    if (ws == nullptr || reinterpret_cast<uintptr_t>(ws) % 256 != 0)
        return fail(TEUK_EINVAL, "the flux workspace must be a 256-byte aligned device pointer");
    if (ws_bytes < 2 * hb)
        return fail(TEUK_ENOMEM, "flux workspace of " + std::to_string(ws_bytes) + " bytes, need " +
                                     std::to_string(2 * hb));
    teuk::FluxParams F;
    F.nmodes = d->nmodes;
    F.nth = d->nth;
    F.rows = d->nsteps + 1;
    F.half_dt = 0.5 * d->dt;
    F.hth = M_PI / (d->nth - 1);
    for (int k = 0; k < d->nmodes; ++k) {
        F.waves[k] = static_cast<const double2*>(d->waves[k]);
        F.m[k] = d->m[k];
        F.next[k] = -1;
        for (int l = 0; l < d->nmodes; ++l)
            if (d->m[l] == d->m[k] + 1) F.next[k] = l;
    }
    F.H = static_cast<double2*>(ws);
    F.K = reinterpret_cast<double2*>(static_cast<char*>(ws) + hb);
    F.out = static_cast<double*>(out);
    HIP_TRY(teuk::launch_flux(F, static_cast<hipStream_t>(hip_stream)), "flux kernels");
    return TEUK_OK;
}

int teuk_set_kernel_timing(teuk_ctx* c, int enable) {
    if (int rc = check_ctx(c)) return rc;
    if (int rc = flush_timing(c)) return rc;
    c->timing = (enable != 0);
    c->timed_ms = 0.0;
    c->timed_launches = 0;
    return TEUK_OK;
}

int teuk_kernel_timing(teuk_ctx* c, double* total_ms, int64_t* launches) {
    if (int rc = check_ctx(c)) return rc;
    if (int rc = flush_timing(c)) return rc;
    if (total_ms) *total_ms = c->timed_ms;
    if (launches) *launches = c->timed_launches;
    return TEUK_OK;
}

int teuk_check_finite(teuk_ctx* c) {
    if (int rc = check_ctx(c)) return rc;
    HIP_TRY(teuk::launch_zero(c->d_flag, sizeof(int), c->stream), "finite flag");
    HIP_TRY(teuk::launch_finite(c->plane[c->cur][0], c->plane[c->cur][1], c->G.nr, c->G.nth, c->ld,
                                c->d_flag, c->stream), "finite kernel");
    int flag = 0;
    HIP_TRY(hipMemcpyAsync(&flag, c->d_flag, sizeof(int), hipMemcpyDeviceToHost, c->stream), "finite copy");
    HIP_TRY(hipStreamSynchronize(c->stream), "finite sync");
    if (flag) return fail(TEUK_ENONFINITE, "state holds NaN or Inf");
    return TEUK_OK;
}

}  // extern "C"
