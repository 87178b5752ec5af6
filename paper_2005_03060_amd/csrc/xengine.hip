// (a4) Reduced X-engine (Fig. 1(b) calibrator box): cross-correlate only the
// antenna pairs of the selected redundant groups,
//     V_ij = (1/T) sum_t v_i(t) conj(v_j(t)),
// on the raw (uncalibrated) voltages.  4-bit voltages are summed exactly in
// int32: |Re q_i conj(q_j)| <= 2*8*8 = 128 per sample, so the sums fit in
// int32 for any T below 2^24.
//
// Antenna-centric: every selected pair (i, j) has r_i - r_j = d_t with d_t
// in the canonical half-plane, so in raster order j = i - (dy n + dx) < i.
// Work-item a owns antenna a and the (at most K) pairs with a first; it
// reads v_a once per sample and its K partners, all from LDS, so a sample
// costs K + 1 LDS reads for K pairs (a pair-centric layout costs 2K).  A
// workgroup owns one unit, one block of B consecutive antennas (B = 512 for
// 4-bit voltages, 256 for complex64) and one
// chunk of samples; each step stages S samples of the antennas
// [a0 - halo, a0 + B) (halo = the largest d_t) with coalesced loads.
// Pairs that do not exist are computed against the antenna itself and
// never written, so the inner loop has no branches.  Partial sums per time
// chunk go to the workspace and a second kernel adds them in a fixed
// order; with a single chunk the first kernel writes V^reduced itself.
//
// 4-bit voltages stay packed (one byte: real part in the high nibble,
// imaginary in the low one) and are multiplied four samples at a time with
// the signed 4-bit dot product (eight nibble products per instruction).  The
// staging transposes 4 x 4 byte blocks so that one LDS word holds four
// consecutive samples of one antenna.  With A the own word and B a
// partner's, dot(A, B) sums ar br + ai bi (the real part).  For the
// imaginary part ai br - ar bi, -ar cannot be formed in 4 bits (-(-8)), but
// -ar = ~ar + 1 and ~ar stays in [-8, 7]: with A' = (ai, ~ar) per byte,
// dot(A', B) = sum ai br + ~ar bi, and adding the partner's own imaginary
// sum (one dot product per antenna, not per pair, exchanged through LDS at
// the end) gives the exact imaginary sum.  Two instructions for four
// samples of one pair, where the unpacked form takes four multiply-adds
// per sample.
// (The int8 matrix-core form for 4-bit voltages is in xmfma.hip; this
// kernel serves complex64 voltages, and 4-bit selections whose window
// cover no matrix-core instantiation holds.)
#include "rrc_device.h"
#include "rrc_launch.h"

#include <type_traits>

namespace rrc {

// Antennas (work-items) per workgroup: 4-bit blocks of 512 halve the share
// of re-read halo antennas against 256 (1.25x the voltages at 64 x 64
// instead of 1.49x; 7.1 -> 6.5 ms there); complex64 keeps 256, whose grids
// then still give enough workgroups without more time chunks.
template <bool CI4>
constexpr int xthreads() { return CI4 ? 512 : 256; }
constexpr int kXHaloMax = 248;   // largest raster offset d_t the staging covers
// LDS row stride of a staged complex64 sample (float2 units), fixed at the
// largest halo: a compile-time stride turns the sample offset of every LDS
// read into an immediate, so the products need no address arithmetic
constexpr int kXRowF = xthreads<false>() + kXHaloMax + 2;
// LDS stride of a staged group of four 4-bit samples (words, one per
// antenna), fixed for the same reason: a group's offset is an immediate
constexpr int kXRowW4 = 1024;
static_assert(kXRowW4 >= xthreads<true>() + kXHaloMax + 6, "a 4-bit group row holds every staged antenna");

// Transpose a 4 x 4 block of bytes: out[k] byte q = in[q] byte k.
__device__ __forceinline__ void transpose4x4(const uint32_t (&w)[4], uint32_t (&o)[4]) {
    // interleave bytes of rows (0, 1) and (2, 3), then 16-bit halves
    const uint32_t t0 = __builtin_amdgcn_perm(w[1], w[0], 0x05010400u);
    const uint32_t t1 = __builtin_amdgcn_perm(w[1], w[0], 0x07030602u);
    const uint32_t t2 = __builtin_amdgcn_perm(w[3], w[2], 0x05010400u);
    const uint32_t t3 = __builtin_amdgcn_perm(w[3], w[2], 0x07030602u);
    o[0] = __builtin_amdgcn_perm(t2, t0, 0x05040100u);
    o[1] = __builtin_amdgcn_perm(t2, t0, 0x07060302u);
    o[2] = __builtin_amdgcn_perm(t3, t1, 0x05040100u);
    o[3] = __builtin_amdgcn_perm(t3, t1, 0x07060302u);
}

// Signed 4-bit dot product of eight nibble pairs, accumulated.
__device__ __forceinline__ int dot8(uint32_t a, uint32_t b, int c) {
    return __builtin_amdgcn_sdot8((int)a, (int)b, c, false);
}

// Samples staged per step: 8 complex64 rows or 64 rows of 4-bit bytes.
template <bool CI4>
constexpr int xeng_samples() { return CI4 ? 64 : 8; }

// Two complex64 values as one 16-byte load (a native vector type, so arrays
// of it stay in registers).
typedef float c64x2 __attribute__((ext_vector_type(4)));

// Antennas per staged load: 4-bit rows move as 32-bit words (4 antennas),
// float rows as 16-byte pairs of antennas when N is even, else singly.
template <bool CI4, bool WIDE>
struct XStage {
    static constexpr int W = CI4 ? 4 : (WIDE ? 2 : 1);
    using RT = typename std::conditional<CI4, uint32_t,
                                         typename std::conditional<WIDE, c64x2, float2>::type>::type;
    static constexpr int KPT = W == 1 ? 2 : 1;   // loads per work-item and row
};

template <bool CI4, bool WIDE, int KMAX>
__global__ __launch_bounds__(xthreads<CI4>(), KMAX <= 9 ? 4 : 2) void k_xant(XengLaunch L) {
    constexpr int NT = xthreads<CI4>();
    constexpr int S = xeng_samples<CI4>();
    using G = XStage<CI4, WIDE>;
    using RT = typename G::RT;
    constexpr int W = G::W, KPT = G::KPT;
    extern __shared__ __align__(16) unsigned char xsm[];

    const int tid = threadIdx.x;
    const int ablk = blockIdx.x;
    const int chunk = blockIdx.y;
    const int unit = blockIdx.z;
    const Sel& s = L.sel;
    const int n = s.n, N = s.N, K = s.K, T = L.T;
    const int a0 = ablk * NT;
    // staged antennas [lo, hi), widened to whole load units (N is a multiple
    // of W on every path)
    const int lo = max(0, a0 - L.halo) / W * W;
    const int hi = (min(N, a0 + NT) + W - 1) / W * W;
    const int cnt = hi - lo;                 // antennas staged per sample
    const int upr = cnt / W;                 // load units per row
    const int a = a0 + tid;
    const bool live = a < N;
    const int ax = a % n, ay = a / n;

    // LDS index of each partner (the antenna itself where the pair does not
    // exist) and the pair's index in V^reduced (-1 if it does not exist)
    int poff[KMAX], pidx[KMAX];
#pragma unroll
    for (int t = 0; t < KMAX; ++t) {
        poff[t] = live ? a - lo : 0;
        pidx[t] = -1;
        if (t >= K || !live) continue;
        const int dx = s.dx[t], dy = s.dy[t];
        const int jx = ax - dx, jy = ay - dy;
        if (jx >= 0 && jx < n && jy >= 0) {
            const int w = n - (dx < 0 ? -dx : dx);
            poff[t] = a - (dy * n + dx) - lo;
            // a masked lattice's table holds -1 where either antenna is absent
            pidx[t] = L.mt.pidx ? L.mt.pidx[(size_t)t * N + a] : s.off[t] + jy * w + (ax - (dx > 0 ? dx : 0));
        }
    }
    const int own = live ? a - lo : 0;

    // float: real and imaginary sums; 4-bit: the real sum and the imaginary
    // one less the partner's own imaginary sum (added at the end)
    using AT = typename std::conditional<CI4, int, float>::type;
    AT accr[KMAX], acci[KMAX];
#pragma unroll
    for (int t = 0; t < KMAX; ++t) accr[t] = acci[t] = 0;
    // 4-bit: sum over the chunk of the imaginary part of antenna a (own) and
    // of halo antenna lo + tid (tid < a0 - lo)
    int sim_own = 0, sim_halo = 0;
    const int hc = a0 - lo;

    const int tb = chunk * L.tchunk;
    const int te = min(T, tb + L.tchunk);

    // Staging: every work-item loads its share of the next S rows into
    // registers (all loads in flight together), then writes them to LDS.
    // Complex64: work-item i copies unit i of every row.  Indices are clamped
    // instead of predicated (a row past the chunk's end repeats the last
    // one, a unit past the row's end repeats the last unit; neither is read),
    // so the copy has no branches.  4-bit: the S rows are S/4 groups of four,
    // and a staging unit is (group g, word column c), four words that are
    // transposed and stored as one 16-byte LDS write: LDS word (g, a) holds
    // samples 4g .. 4g + 3 of antenna a.  Wave w takes groups w, w + 4, ...
    // (row addresses uniform over the wave) and lane l columns l and l + 64,
    // so no word is loaded twice; rows past the chunk's end are zeroed when
    // they go to LDS (not as they arrive, which would wait for each load),
    // since they are summed in groups of four.  4-bit row offsets are
    // 32-bit (at most S rows of N / 4 words).
    const RT* vol = reinterpret_cast<const RT*>(L.volt);
    const size_t rowstride = (size_t)N / W;
    constexpr int NW = NT / 64;
    constexpr int GW = S / 4 / NW;                 // 4-bit groups per wave
    constexpr int CM = ((NT + kXHaloMax + 6) / 4 + 63) / 64;   // word columns per lane
    constexpr int RU = CI4 ? CM * GW : S;          // register rows of staged data
    constexpr int RK = CI4 ? 4 : KPT;
    static_assert(!CI4 || S / 4 % NW == 0, "whole groups per wave");
    RT r[RU][RK];
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6), ln = tid & 63;
    const int rs32 = (int)rowstride;
    int pend_last = S - 1;                         // last valid row of the staged step
    auto load = [&](int t0) {
        const int last = min(S, te - t0) - 1;
        pend_last = last;
        const RT* base = vol + (((size_t)unit * T + t0) * N + lo) / W;
        if constexpr (CI4) {
#pragma unroll
            for (int gi = 0; gi < GW; ++gi) {
                const int g4 = 4 * (wv + NW * gi);
#pragma unroll
                for (int m = 0; m < CM; ++m) {
                    const int c = ln + 64 * m;
                    if (c >= upr) continue;
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const RT* row = base + min(g4 + i, last) * rs32;   // uniform over the wave
                        r[CM * gi + m][i] = row[c];
                    }
                }
            }
        } else {
#pragma unroll
            for (int q = 0; q < S; ++q) {
#pragma unroll
                for (int u = 0; u < KPT; ++u)
                    r[q][u] = base[(size_t)min(q, last) * rowstride + min(tid + u * NT, upr - 1)];
            }
        }
    };
    auto store = [&]() {
        if constexpr (CI4) {
            uint4* st = reinterpret_cast<uint4*>(xsm);
#pragma unroll
            for (int gi = 0; gi < GW; ++gi) {
                const int g = wv + NW * gi;
#pragma unroll
                for (int m = 0; m < CM; ++m) {
                    const int c = ln + 64 * m;
                    if (c >= upr) continue;
                    uint32_t w[4];
#pragma unroll
                    for (int i = 0; i < 4; ++i) w[i] = 4 * g + i <= pend_last ? r[CM * gi + m][i] : 0u;
                    uint32_t o[4];
                    transpose4x4(w, o);
                    st[g * (kXRowW4 / 4) + c] = make_uint4(o[0], o[1], o[2], o[3]);
                }
            }
        } else {
            RT* st = reinterpret_cast<RT*>(xsm);
#pragma unroll
            for (int q = 0; q < S; ++q) {
#pragma unroll
                for (int u = 0; u < KPT; ++u) st[q * (kXRowF / W) + min(tid + u * NT, upr - 1)] = r[q][u];
            }
        }
    };

    if (tb < te) load(tb);
    for (int t0 = tb; t0 < te; t0 += S) {
        const int ns = min(S, te - t0);
        store();
        __syncthreads();
        if (t0 + S < te) load(t0 + S);       // in flight during the products
        // KMAX is the selection's K (or above it, the extra pairs being the
        // antenna with itself, never written): no branch per type
        if constexpr (CI4) {
            // one group: own word and the K partners' words (all reads issued
            // before the products), two dot products per pair
            auto group = [&](const uint32_t* srow) {
                uint32_t vb[KMAX];
                const uint32_t va = srow[own];
                const uint32_t vh = srow[tid];
#pragma unroll
                for (int t = 0; t < KMAX; ++t) vb[t] = srow[poff[t]];
                // (ai, ~ar) per byte: ~ar = -ar - 1 stays in [-8, 7]
                const uint32_t vq = ((va << 4) & 0xF0F0F0F0u) | ((~va >> 4) & 0x0F0F0F0Fu);
                sim_own = dot8(va, 0x01010101u, sim_own);
                sim_halo = dot8(vh, 0x01010101u, sim_halo);
#pragma unroll
                for (int t = 0; t < KMAX; ++t) {
                    accr[t] = dot8(va, vb[t], accr[t]);
                    acci[t] = dot8(vq, vb[t], acci[t]);
                }
            };
            const uint32_t* sw = reinterpret_cast<const uint32_t*>(xsm);
            if (ns == S) {
                // full step: every group's offset is an immediate
#pragma unroll
                for (int g = 0; g < S / 4; ++g) group(sw + g * kXRowW4);
            } else {
                const int ng = (ns + 3) >> 2;
                for (int g = 0; g < ng; ++g) group(sw + g * kXRowW4);
            }
        } else {
            auto products = [&](const float2* srow) {
                const float2 va = srow[own];
#pragma unroll
                for (int t = 0; t < KMAX; ++t) {
                    // two chained FMAs per component: written as one sum of
                    // products, the compiler forms the products' sum first
                    // (a multiply, an FMA and an add)
                    const float2 vb = srow[poff[t]];
                    accr[t] = fmaf(va.x, vb.x, accr[t]);
                    accr[t] = fmaf(va.y, vb.y, accr[t]);
                    acci[t] = fmaf(va.y, vb.x, acci[t]);
                    acci[t] = fmaf(-va.x, vb.y, acci[t]);
                }
            };
            const float2* sb = reinterpret_cast<const float2*>(xsm);
            if (ns == S) {
#pragma unroll
                for (int q = 0; q < S; ++q) products(sb + q * kXRowF);
            } else {
#pragma unroll 2
                for (int q = 0; q < ns; ++q) products(sb + q * kXRowF);
            }
        }
        __syncthreads();
    }

    if constexpr (CI4) {
        // Im(q_i conj q_j) = ai bj_r - ar bj_i and -ar = ~ar + 1, so the
        // imaginary sum is acci plus the partner's own imaginary sum.  The
        // staging buffer is free after the loop's last barrier.
        int* sim = reinterpret_cast<int*>(xsm);
        if (live) sim[own] = sim_own;
        if (tid < hc) sim[tid] = sim_halo;
        __syncthreads();
#pragma unroll
        for (int t = 0; t < KMAX; ++t) acci[t] += sim[poff[t]];
    }

    if (L.nchunk == 1) {
#pragma unroll
        for (int t = 0; t < KMAX; ++t) {
            if (t >= K || pidx[t] < 0) continue;
            const size_t o = (size_t)unit * s.P + pidx[t];
            if constexpr (CI4) reinterpret_cast<int2*>(L.vred)[o] = make_int2(accr[t], acci[t]);
            else reinterpret_cast<float2*>(L.vred)[o] = make_float2(accr[t] * L.inv_t, acci[t] * L.inv_t);
        }
    } else {
        const size_t base = ((size_t)unit * L.nchunk + chunk) * s.P;
#pragma unroll
        for (int t = 0; t < KMAX; ++t) {
            if (t >= K || pidx[t] < 0) continue;
            if constexpr (CI4) reinterpret_cast<int2*>(L.vpart)[base + pidx[t]] = make_int2(accr[t], acci[t]);
            else reinterpret_cast<float2*>(L.vpart)[base + pidx[t]] = make_float2(accr[t], acci[t]);
        }
    }
}

// LDS of one workgroup: complex64, S staged rows of kXRowF values; 4-bit,
// S/4 group rows of kXRowW4 words (up to 512 + halo + 6 antennas, whole
// words, four samples each).
size_t xengine_lds_bytes(int halo, bool ci4) {
    return ci4 ? (size_t)xeng_samples<true>() / 4 * kXRowW4 * 4
               : (size_t)xeng_samples<false>() * kXRowF * 8;
}

int xengine_antennas_per_block(bool ci4) { return ci4 ? xthreads<true>() : xthreads<false>(); }
int xengine_max_halo() { return kXHaloMax; }
int xengine_samples_per_step(bool ci4) { return ci4 ? xeng_samples<true>() : xeng_samples<false>(); }

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

template <bool CI4, bool WIDE, int KMAX>
static hipError_t launch_x(const XengLaunch& L, hipStream_t st) {
    hipError_t e;
    if (CI4 && L.mfma) {
        e = launch_xmfma(L, st);
    } else {
        const size_t lds = xengine_lds_bytes(L.halo, CI4);
        dim3 grid(L.nablk, L.nchunk, L.n_units);
        hipLaunchKernelGGL((k_xant<CI4, WIDE, KMAX>), grid, dim3(xthreads<CI4>()), lds, st, L);
        e = hipGetLastError();
    }
    if (e != hipSuccess || L.nchunk == 1) return e;
    const size_t tot = (size_t)L.n_units * L.sel.P;
    hipLaunchKernelGGL((k_xfin<CI4>), dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, L.vpart,
                       L.nchunk, L.sel.P, L.n_units, L.inv_t, L.vred);
    return hipGetLastError();
}

template <bool CI4, bool WIDE>
static hipError_t launch_x_k(const XengLaunch& L, hipStream_t st) {
    switch (L.sel.K) {
        case 1: case 2: case 3: case 4: case 5: case 6: return launch_x<CI4, WIDE, 6>(L, st);
        case 7: return launch_x<CI4, WIDE, 7>(L, st);
        case 8: return launch_x<CI4, WIDE, 8>(L, st);
        case 9: return launch_x<CI4, WIDE, 9>(L, st);
        case 10: case 11: case 12: return launch_x<CI4, WIDE, 12>(L, st);
        default: return launch_x<CI4, WIDE, kMaxTypes>(L, st);
    }
}

hipError_t launch_xengine(const XengLaunch& L, hipStream_t st) {
    if (L.sel.K < 1 || L.sel.K > kMaxTypes) return hipErrorInvalidValue;
    // staging covers at most 510 antennas per row, in whole words for 4-bit
    if (L.halo > kXHaloMax || (L.ci4 && (L.sel.N & 3))) return hipErrorInvalidValue;
    if (L.tchunk % xengine_samples_per_step(L.ci4)) return hipErrorInvalidValue;
    if (L.ci4) return launch_x_k<true, false>(L, st);
    return (L.sel.N & 1) ? launch_x_k<false, false>(L, st) : launch_x_k<false, true>(L, st);
}

}  // namespace rrc
