// Energy, linear momentum and z angular momentum radiated by the extracted
// waves (the flux and recoil of Sec. 3.2, closing paragraph).  The paper
// prints no formula; the standard psi_4 ones are used, with r psi_4 ->
// sum_m Phi_m(t, theta) e^{i m phi} at the extraction radius (s = -2:
// Psi = rho^-4 psi_4 and the ansatz Psi = e^{i m phi~} r^3 Phi), the news
// integral H = int_0^t r psi_4 dt' and K = int_0^t H dt':
//   dE/dt          = 1/2 sum_m int |H_m|^2 sin dtheta
//   d(Px + i Py)/dt = 1/2 sum_m int H_m conj(H_{m+1}) sin^2 dtheta
//   dPz/dt         = 1/2 sum_m int |H_m|^2 cos sin dtheta
//   dJz/dt         = 1/2 sum_m m Im int conj(H_m) K_m sin dtheta
// (the phi integrals of the definitions done exactly on the Fourier modes),
// time integrals by the trapezoidal rule from t = 0, theta integrals by the
// trapezoidal rule on the rows.
//
// Three launches: the running time integrals of every (mode, row) into the
// workspace (a sequential sum per row: the sum is over time, the rows are
// the parallel dimension); the rates at every time step (one wave per step,
// fixed-order reduction over rows and modes); the accumulated quantities
// (one lane per quantity, sequential over time).
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace teuk {

namespace {

// H and K of row (mode k, theta j): H_0 = 0, H_n = H_{n-1} + (dt/2)(w_{n-1} + w_n),
// and K likewise from H.  Adds and multiplies only (no fma), in the order
// written, so the sums round as the definition reads.
__global__ void flux_integrate_kernel(FluxParams F) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= F.nmodes * F.nth) return;
    const int k = g / F.nth, j = g - k * F.nth;
    const double2* w = F.waves[k] + j;
    double2* H = F.H + static_cast<size_t>(k) * F.rows * F.nth + j;
    double2* K = F.K + static_cast<size_t>(k) * F.rows * F.nth + j;
    const double c = F.half_dt;
    double2 h = make_double2(0.0, 0.0), kk = make_double2(0.0, 0.0);
    double2 wp = w[0];
    H[0] = h;
    K[0] = kk;
    for (int64_t n = 1; n < F.rows; ++n) {
        const double2 wn = w[n * F.nth];
        const double2 hp = h;
        h.x = h.x + c * (wp.x + wn.x);       // no contraction (built with -ffp-contract=off)
        h.y = h.y + c * (wp.y + wn.y);
        kk.x = kk.x + c * (hp.x + h.x);
        kk.y = kk.y + c * (hp.y + h.y);
        H[n * F.nth] = h;
        K[n * F.nth] = kk;
        wp = wn;
    }
}

__device__ inline double wave_sum(double v) {
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// One 64-lane wave per time step n: lane l takes rows l, l + 64, ...
__global__ void __launch_bounds__(256) flux_rates_kernel(FluxParams F) {
    const int64_t n = static_cast<int64_t>(blockIdx.x) * 4 + threadIdx.x / 64;
    const int lane = threadIdx.x % 64;
    if (n >= F.rows) return;
    double e = 0.0, pz = 0.0, px = 0.0, py = 0.0, jz = 0.0;
    for (int k = 0; k < F.nmodes; ++k) {
        const double2* Hk = F.H + (static_cast<size_t>(k) * F.rows + n) * F.nth;
        const double2* Kk = F.K + (static_cast<size_t>(k) * F.rows + n) * F.nth;
        const int k1 = F.next[k];
        const double2* H1 = k1 >= 0 ? F.H + (static_cast<size_t>(k1) * F.rows + n) * F.nth : nullptr;
        const double mk = static_cast<double>(F.m[k]);
        for (int j = lane; j < F.nth; j += 64) {
            double sv, cs;
            sincos(static_cast<double>(j) * F.hth, &sv, &cs);
            const double wq = (j == 0 || j == F.nth - 1) ? 0.5 * F.hth : F.hth;   // trapezoid weight
            const double sn = wq * sv;
            const double2 h = Hk[j], q = Kk[j];
            const double a2 = h.x * h.x + h.y * h.y;
            e += a2 * sn;
            pz += a2 * sn * cs;
            // Im(conj(h) q) = h.x q.y - h.y q.x
            jz += mk * (h.x * q.y - h.y * q.x) * sn;
            if (H1 != nullptr) {
                // h conj(h1) = (h.x h1.x + h.y h1.y) + i (h.y h1.x - h.x h1.y)
                const double2 g = H1[j];
                const double s2 = sn * sv;
                px += (h.x * g.x + h.y * g.y) * s2;
                py += (h.y * g.x - h.x * g.y) * s2;
            }
        }
    }
    e = wave_sum(e);
    pz = wave_sum(pz);
    px = wave_sum(px);
    py = wave_sum(py);
    jz = wave_sum(jz);
    if (lane == 0) {
        double* o = F.out + n * 10;
        o[0] = 0.5 * e;
        o[1] = 0.5 * px;
        o[2] = 0.5 * py;
        o[3] = 0.5 * pz;
        o[4] = 0.5 * jz;
    }
}

// Lane q accumulates quantity q over time by the trapezoidal rule.
__global__ void flux_accumulate_kernel(FluxParams F) {
    const int q = threadIdx.x;
    if (q >= 5) return;
    double acc = 0.0;
    double prev = F.out[q];
    F.out[5 + q] = 0.0;
    for (int64_t n = 1; n < F.rows; ++n) {
        const double cur = F.out[n * 10 + q];
        acc = acc + F.half_dt * (prev + cur);
        F.out[n * 10 + 5 + q] = acc;
        prev = cur;
    }
}

}  // namespace

hipError_t launch_flux(const FluxParams& F, hipStream_t stream) {
    const int rows = F.nmodes * F.nth;
    hipLaunchKernelGGL(flux_integrate_kernel, dim3((rows + 63) / 64), dim3(64), 0, stream, F);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(flux_rates_kernel, dim3(static_cast<unsigned>((F.rows + 3) / 4)), dim3(256), 0, stream, F);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(flux_accumulate_kernel, dim3(1), dim3(64), 0, stream, F);
    return hipGetLastError();
}

}  // namespace teuk
