// Geometry tables of a masked lattice (hexagonal arrays, Sec. 3 and Fig. 2:
// a hexagon in lattice coordinates is a subset of an index grid, and its
// redundant groups are again the pairs at equal displacement).  Rebuilt in
// the caller's workspace from the mask bits, which travel by value in the
// launch descriptor, so a plan owns no device memory.
//
// k_mask_pairs: one workgroup per selected type t.  A pair (a, a - d_t)
// exists when both antennas do; its index in V^reduced is off[t] plus the
// number of existing pairs of the type whose first antenna precedes a in
// raster order (a workgroup prefix count of the existence flags), which is
// the pair order of the reduced visibilities.  Writes pidx[t][a] (or -1)
// and pfirst[b] = a.
// k_mask_lags: the live-antenna bytes, and for every lag d of V^unique the
// group size N_d, counted row by row as popcount(row[y] & (row[y - dy]
// shifted by dx)) with each grid row as a 64-bit mask.
#include "rrc_device.h"
#include "rrc_launch.h"

#include <algorithm>

namespace rrc {

constexpr int kMThr = 256;

__device__ __forceinline__ bool m_live(const MaskLaunch& L, int a) { return (L.bits[a >> 5] >> (a & 31)) & 1u; }

__global__ __launch_bounds__(kMThr) void k_mask_pairs(MaskLaunch L) {
    __shared__ int wcount[kMThr / 64];
    const Sel& s = L.sel;
    const int n = s.n, N = s.N, t = blockIdx.x;
    const int dx = s.dx[t], dy = s.dy[t];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int base = s.off[t];
    for (int a0 = 0; a0 < N; a0 += kMThr) {
        const int a = a0 + tid;
        bool f = false;
        if (a < N) {
            const int ax = a % n, ay = a / n, jx = ax - dx, jy = ay - dy;
            f = m_live(L, a) && jx >= 0 && jx < n && jy >= 0 && m_live(L, jy * n + jx);
        }
        const unsigned long long bal = __ballot(f);
        const int pre = __popcll(bal & ((1ull << lane) - 1ull));
        if (lane == 0) wcount[wave] = __popcll(bal);
        __syncthreads();
        int woff = 0, tot = 0;
        for (int w = 0; w < kMThr / 64; ++w) {
            woff += w < wave ? wcount[w] : 0;
            tot += wcount[w];
        }
        const int idx = base + woff + pre;
        if (a < N) L.pidx[(size_t)t * N + a] = f ? idx : -1;
        if (f) L.pfirst[idx] = a;
        base += tot;
        __syncthreads();   // wcount is rewritten by the next chunk
    }
}

__global__ __launch_bounds__(kMThr) void k_mask_lags(MaskLaunch L) {
    __shared__ unsigned long long row[kMaskGridMax];
    const int n = L.sel.n, N = L.sel.N, tid = threadIdx.x;
    for (int y = tid; y < n; y += kMThr) {
        unsigned long long r = 0ull;
        for (int x = 0; x < n; ++x) r |= (unsigned long long)m_live(L, y * n + x) << x;
        row[y] = r;
    }
    if (blockIdx.x == 0)
        for (int a = tid; a < N; a += kMThr) L.live[a] = m_live(L, a) ? 1 : 0;
    __syncthreads();
    const int nlag = 2 * n * (n - 1);
    for (int l = blockIdx.x * kMThr + tid; l < nlag; l += gridDim.x * kMThr) {
        // lag l in V^unique order: dy = 0, dx = 1 .. n-1; then dy >= 1, dx = -(n-1) .. n-1
        int dx, dy;
        if (l < n - 1) {
            dx = l + 1;
            dy = 0;
        } else {
            const int u = l - (n - 1);
            dy = 1 + u / (2 * n - 1);
            dx = u % (2 * n - 1) - (n - 1);
        }
        int c = 0;
        for (int y = dy; y < n; ++y) {
            const unsigned long long q = dx >= 0 ? row[y - dy] << dx : row[y - dy] >> -dx;
            c += __popcll(row[y] & q);
        }
        L.nd[l] = (float)c;
    }
}

hipError_t launch_mask_tables(const MaskLaunch& L, hipStream_t st) {
    if (L.sel.n > kMaskGridMax || L.sel.K < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_mask_pairs, dim3(L.sel.K), dim3(kMThr), 0, st, L);
    const int nlag = 2 * L.sel.n * (L.sel.n - 1);
    hipLaunchKernelGGL(k_mask_lags, dim3((unsigned)std::max(1, (nlag + kMThr - 1) / kMThr)), dim3(kMThr), 0, st, L);
    return hipGetLastError();
}

}  // namespace rrc
