// Internal state of a context and the library's error helpers, shared by
// the C ABI translation units (capi.cpp, batch.cpp).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/teuk.h"
#include "geometry.h"

namespace teuk_detail {

constexpr int kSourceBatch = 256;   // iterations of source windows per compact pass

extern thread_local std::string g_last_error;
// Record msg as the calling thread's last error and return code.
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);

// Release a context's events and host state and delete it (no ownership
// check); its device memory is the caller's workspace and stays with the caller.
void destroy_ctx(teuk_ctx* c);

// Make the source windows of iteration n resident and return their slot in
// the context's window tables: a source pass over [n, n + nb) (forward) or
// [n - nb + 1, n] (backward), nb = min(span, one source batch), unless the
// resident batch already holds n at amplitude amp.
int ensure_source(teuk_ctx* c, int64_t n, double amp, bool backward, int64_t span, size_t* slot);

#define HIP_TRY(expr, what)                                                  \
    do {                                                                     \
        hipError_t _e = (expr);                                              \
        if (_e != hipSuccess) return teuk_detail::hip_fail(_e, what);        \
    } while (0)

// Byte offsets of a context's device buffers inside its caller-owned
// workspace (every offset a multiple of 256).
struct WsLayout {
    size_t planes = 0;        // 4 state planes: [level][Phi, Pi]
    size_t rnode = 0, rhalf = 0, rows = 0, flag = 0;
    size_t fh = 0, fn = 0, org = 0;        // source windows (win_r_cap x win_t_cap per iteration)
    size_t adj = 0;                        // 4 adjoint planes
    size_t dA = 0, dA_part = 0, dA_blk = 0;
    size_t total = 0;
    int win_r_cap = 0, win_t_cap = 0;      // 0: no room for a source
    bool adjoint = false;
};

// Layout of the workspace for a grid and request; "" or an error message.
std::string ws_layout(const teuk::Geometry& G, int ld, const teuk_ws_request* req, WsLayout* L);

// Context set up on a workspace (no device allocation); on failure nothing is left behind.
int make_ctx(const teuk_grid_desc* d, const teuk_ws_request* req, void* hip_stream, void* ws, size_t ws_bytes,
             teuk_ctx** out);

}  // namespace teuk_detail

struct teuk_ctx {
    teuk::Geometry G;
    bool in_batch = false;          // owned by a teuk_batch: teuk_destroy refuses it
    int static_dev = -1;            // device whose static workspace this context holds (-1: caller's workspace)
    hipStream_t stream = nullptr;
    char* ws = nullptr;             // caller-owned workspace (never freed here)
    teuk_detail::WsLayout lay;
    int ld = 0;
    double2* plane[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};   // [level][Phi, Pi]
    int cur = 0;
    double* d_rnode = nullptr;
    double* d_rhalf = nullptr;
    teuk::ThetaRow* d_rows = nullptr;
    int* d_flag = nullptr;
    double ko_c = 0.0;
    int nstrips = 0, nseg = 0, seg_rows = 16;
    int adj_seg_rows = 4, adj_nseg = 0;   // theta rows per wave segment of the adjoint kernel
    int nsimd = 1024;                     // SIMDs of the device (4 per compute unit)
    int k_steps = 1;               // iterations per stencil launch (temporal blocking depth)
    int bstrips = 0;               // strips of the blocked kernel at depth k_steps
    int64_t steps_done = 0;
    // source
    bool has_src = false;
    double amplitude = 0.0, sig_r = 0.0, sig_th = 0.0, cut = 0.0;
    int64_t nsamples = 0;
    double* d_orbit = nullptr;
    std::vector<double> h_orbit;   // host copy of the orbit (3 per sample)
    int win_r = 0, win_t = 0;
    double2* d_fh = nullptr;
    double2* d_fn = nullptr;
    int4* d_org = nullptr;
    int64_t batch_n0 = -1;
    int batch_len = 0;
    double batch_amp = 0.0;
    // adjoint
    double2* adj[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
    int adj_cur = 0;
    int64_t adj_clock = -1;
    double* d_dA = nullptr;        // accumulated dL/dA (device)
    double* d_dA_part = nullptr;   // per-wave partials of a run of adjoint iterations
    double* d_dA_blk = nullptr;    // block sums of the partials (fixed-order reduction)
    int part_items = 0;            // partials per iteration (waves of the adjoint launch)
    int part_filled = 0;           // iterations written since the last reduction
    // checkpointed gradient (buffers carved from the plan's caller-owned checkpoint buffer)
    double2* snaps = nullptr;      // 2 planes per snapshot: [2k] Phi, [2k+1] Pi, plane_bytes apart
    double2* seg_buf = nullptr;    // Phi on the loss rectangle, one slot per segment iteration
    double* d_ls = nullptr;        // accumulated sum |Phi|^2 over the rectangle
    double* d_ls_part = nullptr;   // per-row partials (nth), then their block sums
    bool ckpt_valid = false;
    teuk_grad_plan ckpt_plan{};
    // kernel timing (measurement aid)
    bool timing = false;
    std::vector<hipEvent_t> ev_start, ev_stop;
    size_t ev_used = 0;
    double timed_ms = 0.0;
    int64_t timed_launches = 0;
};
