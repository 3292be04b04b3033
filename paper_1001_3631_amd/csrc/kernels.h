// Kernel parameter blocks and launchers (internal to the library).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "geometry.h"

namespace teuk {

// Rows of theta per wave segment in the streaming stencil (compiled variants).
constexpr int kSegVariants[] = {4, 8, 16};

// Temporally blocked variants (theta rows per segment, iterations per launch).
struct BlockVariant {
    int seg, k;
};
constexpr BlockVariant kBlockVariants[] = {{4, 2}, {8, 2}, {4, 4}};

struct StepParams {
    const double2* phi;         // u^n planes [nth][ld]
    const double2* pi;
    double2* phi_out;           // u^{n+1} planes
    double2* pi_out;
    const double* rnode;        // radial records, field-major with pitch rpitch
    const double* rhalf;
    const ThetaRow* rows;       // nth angular records
    int nr, nth, ld, rpitch;
    int nstrips, nseg;          // work decomposition: strips of 62 columns x theta segments
    double dt, inv_hr, ko_c;    // ko_c = ko_eps / 16
    int even;                   // |m| even: Neumann poles, else Dirichlet
    int kerr;                   // a != 0
    int i_ext;
    double2* wave;              // nth entries for this iteration, or null
    // source windows of this iteration: both set, or both null when there is
    // no source
    const double2* fh;          // half points: [win_t][win_r]
    const double2* fn;          // nodes: [win_t][win_r]
    const int4* org;            // window origins: half (col0,row0), node (col0,row0)
    int win_r, win_t;
    int frame_first = 0;        // dispatch the general-form waves first (item_order.h)
};

// One instance of a batched launch (homogeneous evolution; see lw_batch_kernel).
struct BatchInstance {
    double2* plane[2][2];       // [level][Phi, Pi], each [nth][ld]
    const double* rnode;
    const double* rhalf;
    const ThetaRow* rows;
    int nr, nth, ld, rpitch;
    int nstrips, nseg;          // tiles (strips) of this instance; theta segments per strip
    double dt, inv_hr, ko_c;
    int even, kerr, i_ext;
    int cur;                    // level holding u at the launch's first iteration
    int tile0;                  // index of its strip 0 in the tile list
    double2* wave;              // [rounds][nth] extraction rows, or null
    // source of the launch's iterations, or all null: iteration n of the
    // launch uses the windows fh + n * win_r * win_t, fn + n * win_r * win_t
    // and the origins org[n]
    const double2* fh;
    const double2* fn;
    const int4* org;
    int win_r, win_t;
};

struct BatchParams {
    const BatchInstance* inst;
    const int4* tiles;          // per tile: (instance, strip, 0, tile index)
    int ntiles;                 // tiles per iteration (all instances)
    int rounds;                 // iterations taken by this launch
    unsigned long long* ticket; // work counter (zero at launch)
    int* done;                  // per tile: iterations completed in this launch (zero at launch)
    int* abort;                 // set to 1 when a dependency wait exceeds wait_limit
    long long wait_limit;       // wall-clock ticks a dependency wait may take
};

struct SourceParams {
    int n0;                     // first iteration (source clock) of the batch
    int4* org;                  // out, per iteration: half (col0,row0), node (col0,row0)
    int win_r, win_t;
    const double* orbit;        // device copy of the orbit samples (3 per sample)
    double amplitude, sig_r, sig_th, cut;
    double rs_min, h_r, h_th;   // grid origin and spacings (window placement)
    int m, nr, nth;
    const double* rnode_rs;     // r* of nodes
    const double* rhalf_rs;     // r* of half points
    const ThetaRow* rows;
    double2* fh;                // output tables, batch-major
    double2* fn;
};

struct PulseParams {
    double2* phi;
    double2* pi;
    int ld, nr, nth, rpitch;
    const double* rnode;
    const double* rnode_rs;
    const ThetaRow* rows;
    double center, width, amplitude;
    int even, kerr;
};

struct AdjointParams {
    // (ordered for a compact argument block: every launch copies it, and a
    // larger block cost 0.2 us per launch on small grids)
    const double2* lam_phi;     // lambda^{n+1} planes [nth][ld]
    const double2* lam_pi;
    double2* out_phi;           // lambda^n planes
    double2* out_pi;
    const double* rnode;        // radial records, pitch nr
    const double* rhalf;
    const ThetaRow* rows;
    int nr, nth, ld;
    int nstrips, nseg;
    int i_ext;
    double dt, inv_hr, ko_c;
    const double2* gw;          // dL/dw_n to inject at column i_ext after the step (nth), or null
    const double2* fh;          // unit-amplitude source windows of the forward iteration n
    const double2* fn;
    const int4* org;
    double* dA_part;            // one partial of dL/dA per wave (nstrips * nseg), or null
    int win_r, win_t;
    // the work items that may meet the source windows: strips [sub_s0,
    // sub_s0 + sub_ns) x segments [sub_g0, sub_g0 + sub_ng) (a superset,
    // from the host's copy of the orbit); the source waves' launch covers
    // only these
    int16_t sub_s0, sub_ns, sub_g0, sub_ng;
    uint8_t even, kerr;
    uint8_t frame_first = 0;    // dispatch the general-form waves first (item_order.h)
};

hipError_t launch_region_sumsq(const double2* phi, int ld, int i0, int i1, int j0, int j1, double* part,
                               hipStream_t stream);
hipError_t launch_add_region(double2* lam, int ld, const double2* src, int src_ld, bool dense, double scale,
                             int i0, int i1, int j0, int j1, hipStream_t stream);

bool valid_segment_rows(int seg);
// nsimd: SIMDs of the device (a launch of more waves than that splits off
// the source waves, see adjoint.hip).
// source_by_window: the windows' rows stay in [3, nth - 4] (no pole folds
// reach them), so the launch may run every wave without source terms and
// take dL/dA from the windows alone (one launch, on any grid).
hipError_t launch_adjoint(const AdjointParams& P, int seg, int nsimd, hipStream_t stream,
                          bool source_by_window = false);
// Whether the rectangle of source items fits its 16-bit fields (P.sub_*).
bool adjoint_rect_fits(int nstrips, int nseg);
// Whether launch_adjoint, when the windows reach the pole rows, runs the
// waves near them in a launch of their own (then it reads P.sub_*).
bool adjoint_splits(int seg, int nstrips, int nseg, int nsimd);
int reduce_partials_blocks(int n);
hipError_t launch_reduce_partials(const double* part, int n, double* blk, double* acc, hipStream_t stream);
hipError_t launch_inject_column(double2* phi, int ld, int nth, int col, const double2* g, hipStream_t stream);
hipError_t launch_add_planes(double2* a, double2* b, const double2* ga, const double2* gb, int nr, int nth,
                             int ld, hipStream_t stream);
hipError_t launch_step(const StepParams& P, int seg, hipStream_t stream, hipEvent_t ev_start = nullptr,
                       hipEvent_t ev_stop = nullptr);
bool valid_block(int seg, int k);
int block_strip_width(int k);
hipError_t launch_block(const StepParams& P, int seg, int k, hipStream_t stream, hipEvent_t ev_start = nullptr,
                        hipEvent_t ev_stop = nullptr);
hipError_t launch_batch_reset(const BatchParams& B, hipStream_t stream);
hipError_t launch_batch(const BatchParams& B, int seg, int waves, hipStream_t stream);
// One iteration n (counted from the table's cur) of the ninst instances of
// inst (a slice of the batch's table); item0 = their first items at segment
// length seg (slice of the batch's offsets, item0[ninst] its end), base =
// item0[0], items = item0[ninst] - base.
hipError_t launch_batch_iteration(const BatchInstance* inst, const int* item0, int ninst, int base, int items,
                                  int n, int seg, hipStream_t stream);
hipError_t launch_source_pass(const SourceParams& S, int nbatch, hipStream_t stream);
hipError_t launch_init_pulse(const PulseParams& Q, hipStream_t stream);
hipError_t launch_finite(const double2* a, const double2* b, int nr, int nth, int ld, int* flag,
                         hipStream_t stream);
// Zero bytes (a multiple of 4) at p (16-byte aligned) on the stream.
hipError_t launch_zero(void* p, size_t bytes, hipStream_t stream);

// Radiated fluxes of the extracted waves (flux.hip).
constexpr int kMaxFluxModes = 16;
struct FluxParams {
    int nmodes = 0, nth = 0;
    int64_t rows = 0;                       // time samples, t = n dt, n = 0 .. rows - 1
    double half_dt = 0.0;
    const double2* waves[kMaxFluxModes] = {};   // [rows][nth] each
    int m[kMaxFluxModes] = {};
    int next[kMaxFluxModes] = {};           // index of the mode with m + 1, or -1
    double hth = 0.0;                       // theta_j = j hth
    double2* H = nullptr;                   // [nmodes][rows][nth]
    double2* K = nullptr;
    double* out = nullptr;                  // [rows][10]
};
hipError_t launch_flux(const FluxParams& F, hipStream_t stream);

// The library's static device workspace (static_ws.hip): its size, and its
// device address on the current device (looked up once per device).
constexpr size_t kStaticWorkspaceBytes = size_t(64) << 20;
hipError_t static_workspace(void** ptr);

}  // namespace teuk
