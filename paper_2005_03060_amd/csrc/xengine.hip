// (a4) Reduced X-engine (Fig. 1(b) calibrator box): cross-correlate only the
// antenna pairs of the selected redundant groups,
//     V_ij = (1/T) sum_t v_i(t) conj(v_j(t)),
// on the raw (uncalibrated) voltages.  4-bit voltages are summed exactly in
// int32: |Re q_i conj(q_j)| <= 2*7*7 = 98 per sample, so 98 * T fits in
// int32 for any T below 2^31 / 98.
//
// A workgroup owns one unit, one chunk of samples and one block of
// NT * PPT pairs.  Each step stages XS samples of the unit's voltages in LDS
// with coalesced loads; every thread then updates its PPT pair accumulators
// from LDS.  Partial sums per time chunk go to the workspace and a second
// kernel adds them in a fixed order.
#include "rrc_device.h"
#include "rrc_launch.h"

namespace rrc {

constexpr int kXThreads = 256;
constexpr int kXLdsBytes = 32768;

__device__ __forceinline__ int2 unpack_ci4(uint8_t b) {
    const int v = b;
    return make_int2((v << 24) >> 28, (v << 28) >> 28);
}

template <int PPT, bool CI4>
__global__ __launch_bounds__(kXThreads) void k_xeng(const void* __restrict__ volt, Sel sel, int T,
                                                    int tchunk, int nchunk, int xs,
                                                    void* __restrict__ vpart) {
    constexpr int NT = kXThreads;
    extern __shared__ __align__(16) unsigned char xsm[];
    const int tid = threadIdx.x;
    const int chunk = blockIdx.x;
    const int pblk = blockIdx.y;
    const int unit = blockIdx.z;
    const int N = sel.N, P = sel.P;
    const int tb = chunk * tchunk;
    const int te = min(T, tb + tchunk);

    int ii[PPT], jj[PPT];
#pragma unroll
    for (int k = 0; k < PPT; ++k) {
        const int p = (pblk * PPT + k) * NT + tid;
        ii[k] = -1;
        jj[k] = 0;
        if (p < P) {
            const int t = type_of(sel, p);
            pair_ij(sel, t, p - sel.off[t], ii[k], jj[k]);
        }
    }

    if constexpr (CI4) {
        int2 acc[PPT];
#pragma unroll
        for (int k = 0; k < PPT; ++k) acc[k] = make_int2(0, 0);
        uint8_t* vs = reinterpret_cast<uint8_t*>(xsm);
        const uint8_t* src = reinterpret_cast<const uint8_t*>(volt) + (size_t)unit * T * N;
        for (int t0 = tb; t0 < te; t0 += xs) {
            const int ns = min(xs, te - t0);
            // stage ns samples (contiguous bytes), 4 bytes per thread-load
            const int nbytes = ns * N;
            const uint8_t* s8 = src + (size_t)t0 * N;
            if ((reinterpret_cast<uintptr_t>(s8) & 3) == 0) {
                const uint32_t* s32 = reinterpret_cast<const uint32_t*>(s8);
                uint32_t* d32 = reinterpret_cast<uint32_t*>(vs);
                for (int q = tid; q < nbytes / 4; q += NT) d32[q] = s32[q];
                for (int q = (nbytes / 4) * 4 + tid; q < nbytes; q += NT) vs[q] = s8[q];
            } else {
                for (int q = tid; q < nbytes; q += NT) vs[q] = s8[q];
            }
            __syncthreads();
            for (int s = 0; s < ns; ++s) {
                const uint8_t* row = vs + s * N;
#pragma unroll
                for (int k = 0; k < PPT; ++k) {
                    if (ii[k] >= 0) {
                        const int2 a = unpack_ci4(row[ii[k]]);
                        const int2 b = unpack_ci4(row[jj[k]]);
                        acc[k].x += a.x * b.x + a.y * b.y;
                        acc[k].y += a.y * b.x - a.x * b.y;
                    }
                }
            }
            __syncthreads();
        }
        int2* out = reinterpret_cast<int2*>(vpart) + ((size_t)unit * nchunk + chunk) * P;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int p = (pblk * PPT + k) * NT + tid;
            if (p < P) out[p] = acc[k];
        }
    } else {
        float2 acc[PPT];
#pragma unroll
        for (int k = 0; k < PPT; ++k) acc[k] = make_float2(0.0f, 0.0f);
        float2* vs = reinterpret_cast<float2*>(xsm);
        const float2* src = reinterpret_cast<const float2*>(volt) + (size_t)unit * T * N;
        for (int t0 = tb; t0 < te; t0 += xs) {
            const int ns = min(xs, te - t0);
            const int nel = ns * N;
            // N is even for every supported grid except odd n; fall back to 8-byte loads then
            if ((N & 1) == 0) {
                const float4* s4 = reinterpret_cast<const float4*>(src + (size_t)t0 * N);
                float4* d4 = reinterpret_cast<float4*>(vs);
                for (int q = tid; q < nel / 2; q += NT) d4[q] = s4[q];
            } else {
                for (int q = tid; q < nel; q += NT) vs[q] = src[(size_t)t0 * N + q];
            }
            __syncthreads();
            for (int s = 0; s < ns; ++s) {
                const float2* row = vs + s * N;
#pragma unroll
                for (int k = 0; k < PPT; ++k) {
                    if (ii[k] >= 0) {
                        const float2 a = row[ii[k]];
                        const float2 b = row[jj[k]];
                        acc[k].x += a.x * b.x + a.y * b.y;
                        acc[k].y += a.y * b.x - a.x * b.y;
                    }
                }
            }
            __syncthreads();
        }
        float2* out = reinterpret_cast<float2*>(vpart) + ((size_t)unit * nchunk + chunk) * P;
#pragma unroll
        for (int k = 0; k < PPT; ++k) {
            const int p = (pblk * PPT + k) * NT + tid;
            if (p < P) out[p] = acc[k];
        }
    }
}

// Sum the time-chunk partials in chunk order; float results are scaled by 1/T.
template <bool CI4>
__global__ __launch_bounds__(256) void k_xfin(const void* __restrict__ vpart, int nchunk, int P,
                                              int n_units, float inv_t, void* __restrict__ vred) {
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (size_t)n_units * P) return;
    const size_t unit = q / P, p = q % P;
    if constexpr (CI4) {
        const int2* src = reinterpret_cast<const int2*>(vpart) + unit * nchunk * P + p;
        int2 s = make_int2(0, 0);
        for (int c = 0; c < nchunk; ++c) {
            const int2 v = src[(size_t)c * P];
            s.x += v.x;
            s.y += v.y;
        }
        reinterpret_cast<int2*>(vred)[q] = s;
    } else {
        const float2* src = reinterpret_cast<const float2*>(vpart) + unit * nchunk * P + p;
        float2 s = make_float2(0.0f, 0.0f);
        for (int c = 0; c < nchunk; ++c) s = cadd(s, src[(size_t)c * P]);
        reinterpret_cast<float2*>(vred)[q] = make_float2(s.x * inv_t, s.y * inv_t);
    }
}

template <int PPT, bool CI4>
static hipError_t launch_x(const XengLaunch& L, hipStream_t st) {
    const size_t lds = (size_t)L.xs * L.sel.N * (CI4 ? 1 : 8);
    dim3 grid(L.nchunk, L.npblk, L.n_units);
    hipLaunchKernelGGL((k_xeng<PPT, CI4>), grid, dim3(kXThreads), lds, st, L.volt, L.sel, L.T,
                       L.tchunk, L.nchunk, L.xs, L.vpart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t tot = (size_t)L.n_units * L.sel.P;
    hipLaunchKernelGGL((k_xfin<CI4>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, L.vpart,
                       L.nchunk, L.sel.P, L.n_units, 1.0f / (float)L.T, L.vred);
    return hipGetLastError();
}

hipError_t launch_xengine(const XengLaunch& L, hipStream_t st) {
    switch (L.ppt) {
        case 4: return L.ci4 ? launch_x<4, true>(L, st) : launch_x<4, false>(L, st);
        case 8: return L.ci4 ? launch_x<8, true>(L, st) : launch_x<8, false>(L, st);
        case 16: return L.ci4 ? launch_x<16, true>(L, st) : launch_x<16, false>(L, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace rrc
