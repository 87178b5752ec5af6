// (a4) Reduced X-engine for 4-bit voltages on the int8 matrix cores
// (Fig. 1(b) calibrator box; Sec. 5 subset selection): for every selected
// pair, S_ij = sum_t q_i(t) conj(q_j(t)) exactly in int32.
//
// The product over the time axis is a dense complex matrix product, so it
// runs as v_mfma_i32_16x16x64_i8 tiles: rows are a block of 16 consecutive
// antennas i (raster order), columns a window of 16 consecutive antennas j,
// k the samples.  A selected pair has j = i - d_t with d_t = dy n + dx the
// type's raster offset, so for a row block starting at r0 the partners lie
// in the union over t of [r0 - d_t, r0 + 15 - d_t]; the plan covers that
// union with windows [r0 + c, r0 + c + 16) (the same offsets c for every
// row block) and runs of windows 16 apart.  A wave owns two consecutive
// row blocks, so a run of L windows needs L + 1 column loads, not 2L.
// Only the entries on the selected diagonals of each tile are kept.
//
// Operands.  Each staged sample of antenna a is expanded to three int8
// planes, R = 8 re, S = 8 im and S' = -8 im (a nibble's -8 becomes -64, and
// -(-64) = 64 still fits int8).  One 16x16x64 product covers 32 samples,
// its K = 64 slots taken as two halves of 32.  Per lane group g = lane / 16
// (the group's k slots) the operands are
//     re: A = R_i / S_i (g < 2 / g >= 2),  B = R_j / S_j
//     im: A = S_i / R_i,                   B = R_j / S'_j
// (g even / odd: samples 0-15 / 16-31 of the step), so
//     acc_re = 64 sum (ar ar' + ai ai') = 64 Re(q_i conj q_j),
//     acc_im = 64 sum (ai ar' - ar ai') = 64 Im(q_i conj q_j).
// A and B read their k slots with the same rule, so the result does not
// depend on the order in which the hardware walks k.  |acc| <= 64 * 128 * T
// per time chunk: exact in int32 for chunks below 2^18 samples.
//
// Staging: 32 samples per step of the antennas the workgroup's windows
// reach, loaded as 32-bit words (four antennas of one sample), transposed
// in 4 x 4 byte blocks (one word = four samples of one antenna), split into
// the three planes and stored antenna-major: 112 bytes per antenna
// (R, S, S' of 32 samples and 16 bytes of padding), which makes the
// 16-byte operand reads of 16 consecutive antennas fall in distinct banks.
// The next step's words are loaded into registers while the current one is
// multiplied.
#include "rrc_device.h"
#include "rrc_launch.h"

#include <algorithm>
#include <vector>

namespace rrc {

typedef int v4i __attribute__((ext_vector_type(4)));

constexpr int kMThreads = 512;              // 8 waves
constexpr int kMRowsPerWave = 32;           // two row blocks of 16
constexpr int kMAntPerGroup = kMThreads / 64 * kMRowsPerWave;   // 256 rows per workgroup
constexpr int kMStep = 32;                  // samples per staged step
constexpr int kMStride = 112;               // LDS bytes per staged antenna
constexpr int kMMaxChunk = 1 << 17;         // samples per chunk: int32 exact below 2^18

// 4 x 4 byte transpose: out[k] byte q = in[q] byte k.
__device__ __forceinline__ void xm_transpose4x4(const uint32_t (&w)[4], uint32_t (&o)[4]) {
    const uint32_t t0 = __builtin_amdgcn_perm(w[1], w[0], 0x05010400u);
    const uint32_t t1 = __builtin_amdgcn_perm(w[1], w[0], 0x07030602u);
    const uint32_t t2 = __builtin_amdgcn_perm(w[3], w[2], 0x05010400u);
    const uint32_t t3 = __builtin_amdgcn_perm(w[3], w[2], 0x07030602u);
    o[0] = __builtin_amdgcn_perm(t2, t0, 0x05040100u);
    o[1] = __builtin_amdgcn_perm(t2, t0, 0x07060302u);
    o[2] = __builtin_amdgcn_perm(t3, t1, 0x05040100u);
    o[3] = __builtin_amdgcn_perm(t3, t1, 0x07060302u);
}

// Four packed bytes (re << 4 | im) -> 8 re, 8 im, -8 im as packed int8.
// x & 0xF0 is 16 re; an arithmetic halving per byte keeps the sign bit
// (the bit shifted in from the byte above is a masked-off zero).
__device__ __forceinline__ void xm_planes(uint32_t w, uint32_t& r, uint32_t& s, uint32_t& sn) {
    const uint32_t hr = w & 0xF0F0F0F0u;              // 16 re per byte
    const uint32_t hi = (w << 4) & 0xF0F0F0F0u;       // 16 im per byte
    r = (hr >> 1) | (hr & 0x80808080u);
    s = (hi >> 1) | (hi & 0x80808080u);
    // per-byte negation of s in two 16-bit lanes (no borrow crosses a byte:
    // 0x100 - v >= 1 for every byte value v)
    const uint32_t ev = s & 0x00FF00FFu, od = (s >> 8) & 0x00FF00FFu;
    sn = ((0x01000100u - ev) & 0x00FF00FFu) | (((0x01000100u - od) & 0x00FF00FFu) << 8);
}

__device__ __forceinline__ v4i lds_v4(const unsigned char* p) { return *reinterpret_cast<const v4i*>(p); }

template <int NR, int L>
__global__ __launch_bounds__(kMThreads) void k_xmfma(XengLaunch X) {
    constexpr int RW = 2;
    extern __shared__ __align__(16) unsigned char msm[];
    const Sel& s = X.sel;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int unit = blockIdx.z, chunk = blockIdx.y;
    const int N = s.N, T = X.T;
    const int a0 = blockIdx.x * kMAntPerGroup;
    const int lo = a0 + X.mf_lo;                 // first staged antenna (4-aligned offset)
    const int cnt = X.mf_cnt;                    // staged antennas (multiple of 4)
    const int tb = chunk * X.tchunk, te = min(T, tb + X.tchunk);

    // ---- staging: (word column m, 4-sample group q) blocks, at most two
    // per work-item
    const int nwc = cnt >> 2;
    const int nblk = nwc * (kMStep / 4);
    const uint32_t* vol = reinterpret_cast<const uint32_t*>(X.volt);
    const size_t row_words = (size_t)N >> 2;
    uint32_t pre[2][4];
    auto load = [&](int t0) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int blk = tid + h * kMThreads;
            const int m = blk % nwc, q = blk / nwc;
            const int a = lo + 4 * m;
            const bool in = blk < nblk && a >= 0 && a < N;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int t = t0 + 4 * q + r;
                pre[h][r] = (in && t < te) ? vol[((size_t)unit * T + t) * row_words + (a >> 2)] : 0u;
            }
        }
    };
    auto store = [&]() {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int blk = tid + h * kMThreads;
            if (blk >= nblk) continue;
            const int m = blk % nwc, q = blk / nwc;
            uint32_t o[4];
            xm_transpose4x4(pre[h], o);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                uint32_t r, sv, sn;
                xm_planes(o[e], r, sv, sn);
                unsigned char* p = msm + (4 * m + e) * kMStride + 4 * q;
                *reinterpret_cast<uint32_t*>(p) = r;
                *reinterpret_cast<uint32_t*>(p + 32) = sv;
                *reinterpret_cast<uint32_t*>(p + 64) = sn;
            }
        }
    };

    // ---- this lane's operand offsets
    const int g = lane >> 4, li = lane & 15;
    const int off_re = 16 * g;                              // [R | S]
    const int off_aim = (16 * g + 32) & 63;                 // [S | R]
    const int off_bim = 16 * g + (g >= 2 ? 32 : 0);         // [R | S']
    const int rw0 = a0 + wave * kMRowsPerWave;              // first row of the wave
    v4i acc_re[NR][RW][L], acc_im[NR][RW][L];
#pragma unroll
    for (int r = 0; r < NR; ++r)
#pragma unroll
        for (int b = 0; b < RW; ++b)
#pragma unroll
            for (int m = 0; m < L; ++m) {
                acc_re[r][b][m] = v4i{0, 0, 0, 0};
                acc_im[r][b][m] = v4i{0, 0, 0, 0};
            }

    if (tb < te) load(tb);
    for (int t0 = tb; t0 < te; t0 += kMStep) {
        store();
        __syncthreads();
        if (t0 + kMStep < te) load(t0 + kMStep);           // in flight during the products
        v4i are[RW], aim[RW];
#pragma unroll
        for (int b = 0; b < RW; ++b) {
            const unsigned char* p = msm + (rw0 + 16 * b + li - lo) * kMStride;
            are[b] = lds_v4(p + off_re);
            aim[b] = lds_v4(p + off_aim);
        }
#pragma unroll
        for (int r = 0; r < NR; ++r) {
            if (r >= X.mf_nrun) break;
            const int c0 = rw0 + X.mf_start[r] + li - lo;   // column of window u = 0
            const int lr = X.mf_len[r];
#pragma unroll
            for (int u = 0; u < RW + L - 1; ++u) {
                if (u >= RW + lr - 1) break;
                const unsigned char* p = msm + (c0 + 16 * u) * kMStride;
                const v4i bre = lds_v4(p + off_re);
                const v4i bim = lds_v4(p + off_bim);
#pragma unroll
                for (int b = 0; b < RW; ++b) {
                    const int m = u - b;
                    if (m < 0 || m >= L) continue;
                    if (m >= lr) continue;
                    acc_re[r][b][m] = __builtin_amdgcn_mfma_i32_16x16x64_i8(are[b], bre, acc_re[r][b][m], 0, 0, 0);
                    acc_im[r][b][m] = __builtin_amdgcn_mfma_i32_16x16x64_i8(aim[b], bim, acc_im[r][b][m], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }

    // ---- the selected diagonals: lane holds rows 4g .. 4g+3 of column li
    int2* out = reinterpret_cast<int2*>(X.nchunk == 1 ? X.vred : X.vpart);
    const size_t obase = X.nchunk == 1 ? (size_t)unit * s.P : ((size_t)unit * X.nchunk + chunk) * s.P;
#pragma unroll
    for (int r = 0; r < NR; ++r) {
        if (r >= X.mf_nrun) break;
#pragma unroll
        for (int b = 0; b < RW; ++b) {
#pragma unroll
            for (int m = 0; m < L; ++m) {
                if (m >= X.mf_len[r]) continue;
                const int j = rw0 + 16 * b + X.mf_start[r] + 16 * m + li;   // column antenna
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int i = rw0 + 16 * b + 4 * g + e;                   // row antenna
                    if (i >= N || j < 0) continue;
                    const int d = i - j;
                    const int ax = i % s.n, ay = i / s.n;
                    for (int t = 0; t < s.K; ++t) {
                        const int dx = s.dx[t], dy = s.dy[t];
                        if (dy * s.n + dx != d) continue;
                        const int jx = ax - dx, jy = ay - dy;
                        if (jx < 0 || jx >= s.n || jy < 0) continue;
                        const int w = s.n - (dx < 0 ? -dx : dx);
                        const int pidx = s.off[t] + jy * w + (ax - (dx > 0 ? dx : 0));
                        out[obase + pidx] = make_int2(acc_re[r][b][m][e] >> 6, acc_im[r][b][m][e] >> 6);
                    }
                }
            }
        }
    }
}

// The window cover of a selection (see the file comment): runs of windows
// 16 apart, as offsets from a row block's first antenna.  Returns false if
// it needs more runs or longer runs than any instantiation holds.
bool xmfma_plan(const Sel& s, XengLaunch& X) {
    std::vector<int> vals;
    for (int t = 0; t < s.K; ++t) {
        const int d = s.dy[t] * s.n + s.dx[t];
        for (int v = -d; v < 16 - d; ++v) vals.push_back(v);
    }
    std::sort(vals.begin(), vals.end());
    vals.erase(std::unique(vals.begin(), vals.end()), vals.end());
    std::vector<int> wins;
    for (size_t i = 0; i < vals.size();) {
        const int st = vals[i];
        wins.push_back(st);
        while (i < vals.size() && vals[i] < st + 16) ++i;
    }
    int nrun = 0, start[kXMaxRuns] = {0}, len[kXMaxRuns] = {0};
    for (int w : wins) {
        if (nrun > 0 && start[nrun - 1] + 16 * len[nrun - 1] == w) {
            ++len[nrun - 1];
        } else {
            if (nrun == kXMaxRuns) return false;
            start[nrun] = w;
            len[nrun] = 1;
            ++nrun;
        }
    }
    int lmax = 0;
    for (int r = 0; r < nrun; ++r) lmax = std::max(lmax, len[r]);
    // instantiations (runs, run length): (1,2) (1,3) (1,5) (2,3) (3,2) (3,3)
    int inst = -1;
    const int nr_of[6] = {1, 1, 1, 2, 3, 3}, l_of[6] = {2, 3, 5, 3, 2, 3};
    for (int k = 0; k < 6; ++k) {
        if (nr_of[k] < nrun || l_of[k] < lmax) continue;
        if (inst < 0 || nr_of[k] * l_of[k] < nr_of[inst] * l_of[inst]) inst = k;
    }
    if (inst < 0) return false;
    // staged antennas of a workgroup, relative to its first row a0: its
    // rows [0, 256) and every window's columns [16 b + w, 16 b + w + 16)
    // for row blocks b < 16, i.e. [min(w, 0), 256 + max(w, 0))
    const int wmin = std::min(wins.front(), 0), wmax = std::max(wins.back(), 0);
    const int lo = (wmin >= 0 ? wmin / 4 : -((-wmin + 3) / 4)) * 4;
    const int hi = kMAntPerGroup + wmax;
    // the staging copies (word column, 4-sample group) blocks, at most two
    // per work-item
    if ((hi - lo + 3) / 4 * (kMStep / 4) > 2 * kMThreads) return false;
    X.mf_inst = inst;
    X.mf_nrun = nrun;
    for (int r = 0; r < kXMaxRuns; ++r) {
        X.mf_start[r] = start[r];
        X.mf_len[r] = len[r];
    }
    X.mf_lo = lo;
    X.mf_cnt = (hi - lo + 3) / 4 * 4;
    return true;
}

size_t xmfma_lds_bytes(const XengLaunch& X) { return (size_t)X.mf_cnt * kMStride; }
int xmfma_antennas_per_group() { return kMAntPerGroup; }
int xmfma_step() { return kMStep; }
int xmfma_max_chunk() { return kMMaxChunk; }

template <int NR, int L>
static hipError_t launch_m(const XengLaunch& X, hipStream_t st) {
    dim3 grid((X.sel.N + kMAntPerGroup - 1) / kMAntPerGroup, X.nchunk, X.n_units);
    hipLaunchKernelGGL((k_xmfma<NR, L>), grid, dim3(kMThreads), xmfma_lds_bytes(X), st, X);
    return hipGetLastError();
}

hipError_t launch_xmfma(const XengLaunch& X, hipStream_t st) {
    if (X.tchunk % kMStep || X.tchunk > kMMaxChunk || (X.sel.N & 3)) return hipErrorInvalidValue;
    switch (X.mf_inst) {
        case 0: return launch_m<1, 2>(X, st);
        case 1: return launch_m<1, 3>(X, st);
        case 2: return launch_m<1, 5>(X, st);
        case 3: return launch_m<2, 3>(X, st);
        case 4: return launch_m<3, 2>(X, st);
        case 5: return launch_m<3, 3>(X, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace rrc
