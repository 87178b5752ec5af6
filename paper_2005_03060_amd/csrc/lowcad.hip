// Low-cadence calibration (Sec. 4): the calibrator correlates about
// p N log N baselines at a time (eq. lowcadcal_inttime) and cycles through
// every redundant group, whole groups per cycle; after N_cycle cycles of
// t_int = t_cal / N_cycle each, the populated visibility matrix is
// calibrated once, over every type.
//
// Schedule (host): groups in V^unique's lag order, a cycle taking whole
// groups while its pair count stays within p N ln N, so cycle c is a range
// of lag-order types and of the all-type pair list; it integrates samples
// [c T / N_cycle, (c + 1) T / N_cycle) of the interval.
// X-engine (k_xlowcad): one work-item per pair of the all-type list (type
// major in lag order, then the raster index of the first antenna), summing
// v_i conj(v_j) over its cycle's samples in FP32; consecutive work-items
// hold consecutive first antennas of one type, so each sample's loads of
// v_i and v_j are contiguous runs.  The solve is the omnical iteration over
// every type (omnical.hip).
#include "rrc_device.h"
#include "rrc_launch.h"

#include <algorithm>
#include <cmath>
#include <vector>

#include "../../include/rrcal.h"

namespace rrc {

constexpr int kLThreads = 256;
static_assert(kLowcadMaxCycles == RRC_LOWCAD_MAX_CYCLES, "cycle bound of the launch descriptor");

// pairs before lag-order type (dx, dy) of an n x n grid
__device__ __forceinline__ long l_off(int n, int dx, int dy) {
    const long N = (long)n * n;
    if (dy == 0) {
        const long m = dx - 1;                             // sum_{k=1}^{m} (n - k) rows of n
        return (long)n * (m * n - m * (m + 1) / 2);
    }
    const long base = (long)n * ((long)n * (n - 1) / 2);   // every dy = 0 type
    const long r = dy - 1;
    const long rows = N * (r * n - r * (r + 1) / 2);       // rows dy' = 1 .. dy-1, n^2 (n - dy') each
    long f;                                                // sum_{d=-(n-1)}^{dx-1} (n - |d|)
    if (dx <= 0) f = (long)(n + dx - 1) * (n + dx) / 2;
    else f = (long)n * (n - 1) / 2 + (long)dx * n - (long)dx * (dx - 1) / 2;
    return base + rows + (n - dy) * f;
}

__device__ __forceinline__ void l_lag(int n, int t, int& dx, int& dy) {
    if (t < n - 1) {
        dx = t + 1;
        dy = 0;
    } else {
        const int u = t - (n - 1);
        dy = 1 + u / (2 * n - 1);
        dx = u % (2 * n - 1) - (n - 1);
    }
}

__global__ __launch_bounds__(kLThreads) void k_xlowcad(LowcadLaunch L) {
    const int n = L.n, N = n * n, K = 2 * n * (n - 1);
    const long P = (long)N * (N - 1) / 2;
    const long b = (long)blockIdx.x * kLThreads + threadIdx.x;
    const int unit = blockIdx.y;
    if (b >= P) return;
    // type of pair b: the last lag-order type whose offset is <= b
    int lo = 0, hi = K - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        int dx, dy;
        l_lag(n, mid, dx, dy);
        if (l_off(n, dx, dy) <= b) lo = mid;
        else hi = mid - 1;
    }
    int dx, dy;
    l_lag(n, lo, dx, dy);
    const int bl = (int)(b - l_off(n, dx, dy));
    const int w = n - (dx < 0 ? -dx : dx);
    const int i = (bl / w + dy) * n + bl % w + (dx > 0 ? dx : 0), j = i - (dy * n + dx);
    // its cycle: the last cycle whose first type is <= the pair's type
    int c = 0;
    while (c + 1 < L.n_cycles && L.type_begin[c + 1] <= lo) ++c;
    const int s0 = (int)((long)c * L.T / L.n_cycles), s1 = (int)((long)(c + 1) * L.T / L.n_cycles);
    const float2* v = reinterpret_cast<const float2*>(L.volt) + (size_t)unit * L.T * N;
    float2 acc = make_float2(0.f, 0.f);
    for (int s = s0; s < s1; ++s) {
        const float2 a = v[(size_t)s * N + i], q = v[(size_t)s * N + j];
        acc.x = fmaf(a.x, q.x, fmaf(a.y, q.y, acc.x));
        acc.y = fmaf(a.y, q.x, fmaf(-a.x, q.y, acc.y));
    }
    const float inv = 1.0f / (float)(s1 - s0);
    reinterpret_cast<float2*>(L.vfull)[(size_t)unit * P + b] = make_float2(acc.x * inv, acc.y * inv);
}

// Whole-array fit of the FFT-correlator's model (Sec. 2 scatter of
// redundant visibilities; Sec. 6.4): for every pair of the all-type list,
// r = V_ij - g_i conj(g_j) V^unique(d_ij), summed in FP64 as |r|^2 (eq. redchi
// with sigma = 1) and as |r / (g_i conj(g_j))|^2 (the calibrated residual,
// whose noise is the same for every pair).  One workgroup per unit, types in
// lag order (the all-type list's order and V^unique's), a fixed reduction
// order.
__global__ __launch_bounds__(kLThreads) void k_chisq_full(int n, const float2* __restrict__ vfull,
                                                          const float2* __restrict__ gains,
                                                          const float2* __restrict__ vunique,
                                                          double* __restrict__ chisq,
                                                          double* __restrict__ chisq_cal) {
    __shared__ double red[2][kLThreads / 64];
    const int N = n * n, K = 2 * n * (n - 1), unit = blockIdx.x, tid = threadIdx.x;
    const long P = (long)N * (N - 1) / 2;
    const float2* vf = vfull + (size_t)unit * P;
    const float2* g = gains + (size_t)unit * N;
    const float2* vu = vunique + (size_t)unit * K;
    double s = 0.0, sc = 0.0;
    long off = 0;
    for (int t = 0; t < K; ++t) {
        int dx, dy;
        l_lag(n, t, dx, dy);
        const int w = n - (dx < 0 ? -dx : dx), cnt = w * (n - dy);
        const double2 va = make_double2(vu[t].x, vu[t].y);
        for (int b = tid; b < cnt; b += kLThreads) {
            const int i = (b / w + dy) * n + b % w + (dx > 0 ? dx : 0), j = i - (dy * n + dx);
            const double gr = (double)g[i].x * g[j].x + (double)g[i].y * g[j].y;   // g_i conj(g_j)
            const double gim = (double)g[i].y * g[j].x - (double)g[i].x * g[j].y;
            const double mr = gr * va.x - gim * va.y, mi = gr * va.y + gim * va.x;
            const double rr = (double)vf[off + b].x - mr, ri = (double)vf[off + b].y - mi;
            const double e2 = rr * rr + ri * ri;
            s += e2;
            sc += e2 / (gr * gr + gim * gim);
        }
        off += cnt;
    }
    for (int o = 1; o < 64; o <<= 1) {
        s += __shfl_xor(s, o, 64);
        sc += __shfl_xor(sc, o, 64);
    }
    if ((tid & 63) == 0) {
        red[0][tid >> 6] = s;
        red[1][tid >> 6] = sc;
    }
    __syncthreads();
    if (tid == 0) {
        double a = 0.0, c = 0.0;
        for (int w = 0; w < kLThreads / 64; ++w) {
            a += red[0][w];
            c += red[1][w];
        }
        chisq[unit] = a;
        if (chisq_cal) chisq_cal[unit] = c;
    }
}

hipError_t launch_xlowcad(const LowcadLaunch& L, hipStream_t st) {
    const long P = (long)L.n * L.n * ((long)L.n * L.n - 1) / 2;
    hipLaunchKernelGGL(k_xlowcad, dim3((unsigned)((P + kLThreads - 1) / kLThreads), L.n_units), dim3(kLThreads),
                       0, st, L);
    return hipGetLastError();
}

}  // namespace rrc

extern "C" {

int rrc_lowcad_schedule(int32_t n, double p, double log_base, int32_t* type_begin, int32_t cap,
                        int32_t* n_cycles) {
    if (n < 2 || n > RRC_MAX_GRID || !(p > 0.0) || !type_begin || !n_cycles || cap < 1) return RRC_EINVAL;
    const double N = (double)n * n;
    const double lg = (log_base > 1.0) ? std::log(N) / std::log(log_base) : std::log(N);
    const double budget = p * N * lg;
    const int K = 2 * n * (n - 1);
    int nc = 0;
    long cnt = 0;
    for (int t = 0; t < K; ++t) {
        int dx, dy;
        if (t < n - 1) {
            dx = t + 1;
            dy = 0;
        } else {
            dy = 1 + (t - (n - 1)) / (2 * n - 1);
            dx = (t - (n - 1)) % (2 * n - 1) - (n - 1);
        }
        const long m = (long)(n - std::abs(dx)) * (n - dy);
        if (t == 0 || (cnt > 0 && (double)(cnt + m) > budget)) {
            if (nc == cap) return RRC_ERANGE;
            type_begin[nc++] = t;
            cnt = 0;
        }
        cnt += m;
    }
    if (nc >= cap) return RRC_ERANGE;
    type_begin[nc] = K;
    *n_cycles = nc;
    return RRC_OK;
}

int rrc_lowcad_xengine(int32_t n, int32_t n_units, int32_t n_time, const int32_t* type_begin,
                       int32_t n_cycles, void* stream, const void* d_volt, void* d_vfull) {
    if (n < 2 || n > RRC_LOWCAD_MAX_GRID || n_units < 1 || n_cycles < 1 || n_cycles > RRC_LOWCAD_MAX_CYCLES ||
        n_time < n_cycles || !type_begin || !d_volt || !d_vfull)
        return RRC_EINVAL;
    const int K = 2 * n * (n - 1);
    if (type_begin[0] != 0 || type_begin[n_cycles] != K) return RRC_EINVAL;
    for (int c = 0; c < n_cycles; ++c)
        if (type_begin[c + 1] <= type_begin[c]) return RRC_EINVAL;
    rrc::LowcadLaunch L{};
    L.n = n;
    L.n_units = n_units;
    L.T = n_time;
    L.n_cycles = n_cycles;
    for (int c = 0; c <= n_cycles; ++c) L.type_begin[c] = type_begin[c];
    L.volt = d_volt;
    L.vfull = d_vfull;
    return rrc::launch_xlowcad(L, reinterpret_cast<hipStream_t>(stream)) == hipSuccess ? RRC_OK : RRC_EDEVICE;
}

int rrc_chisq_full(int32_t n, int32_t n_units, void* stream, const void* d_vfull, const void* d_gains,
                   const void* d_vunique, double* d_chisq, double* d_chisq_cal) {
    if (n < 2 || n > RRC_LOWCAD_MAX_GRID || n_units < 1 || !d_vfull || !d_gains || !d_vunique || !d_chisq)
        return RRC_EINVAL;
    hipLaunchKernelGGL(rrc::k_chisq_full, dim3(n_units), dim3(rrc::kLThreads), 0,
                       reinterpret_cast<hipStream_t>(stream), n, static_cast<const float2*>(d_vfull),
                       static_cast<const float2*>(d_gains), static_cast<const float2*>(d_vunique), d_chisq,
                       d_chisq_cal);
    return hipGetLastError() == hipSuccess ? RRC_OK : RRC_EDEVICE;
}

int rrc_lowcad_solve(int32_t n, int32_t n_units, void* stream, const void* d_vfull, const void* d_gains_in,
                     int32_t max_iter, float tol, void* d_gains, void* d_vmodel, float* d_chisq,
                     int32_t* d_niter, int32_t* d_status) {
    if (n < 3 || n > RRC_LOWCAD_MAX_GRID || n_units < 1 || !d_vfull || !d_gains_in || !d_gains || !d_vmodel ||
        !d_chisq || !d_niter || !d_status || max_iter < 1 || !(tol >= 0.f))
        return RRC_EINVAL;
    rrc::OmniLaunch L{};
    L.n = n;
    L.K = 2 * n * (n - 1);
    L.P = n * n * (n * n - 1) / 2;
    L.n_units = n_units;
    L.all = true;
    L.ci4 = false;
    L.lds_types = (((size_t)3 * L.K + 1) * 4 + 15) / 16 * 16;
    L.max_iter = max_iter;
    L.tol = tol;
    L.damping = 0.3f;
    L.finish = true;
    L.gains_in = reinterpret_cast<const float2*>(d_gains_in);
    L.vred = d_vfull;
    L.gains = d_gains;
    L.vmodel = d_vmodel;
    L.chisq = d_chisq;
    L.niter = d_niter;
    L.status = d_status;
    L.delta = nullptr;
    return rrc::launch_omnical(L, reinterpret_cast<hipStream_t>(stream)) == hipSuccess ? RRC_OK : RRC_EDEVICE;
}

}  // extern "C"
