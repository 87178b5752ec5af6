// (a1)-(a3) FFT-correlator: gain application, zero-padded 2-D spatial FFT
// per sample, |E|^2 integrated over time, inverse transform and redundant
// normalisation (Fig. 1(b) yellow box; eq. modelvis; convolution theorem of
// Sec. 1).
//
// Pass 1 (k_fftcorr): one workgroup owns one unit and one chunk of samples.
// It processes S samples per step.  Row stage: thread (s, y, h) loads row y
// of sample s (n voltages) straight from HBM, divides by the gains, and
// computes the h-th half of that row's M-point transform: because only the
// first n <= M/2 inputs are non-zero, E(2m) is the M/2-point FFT of x_k and
// E(2m+1) the M/2-point FFT of x_k w_M^k, so each half is independent.  The
// halves go to an LDS row buffer.  Column stage: thread (u, h') takes column
// u of two samples and does the same half-split transform over y, squaring
// and accumulating |E|^2 in registers across the whole chunk.  Partial power
// grids are reduced in LDS and written once per workgroup.
//
// Finish (a second kernel, one workgroup per unit): sum the unit's partial
// grids in a fixed order and transform back,
// C(d) = (1/M^2) sum_u P(u) e^{+2 pi i u.d/M}, then V(d) = C(d) / (N_d T).
// For M <= 64 with register FFTs (k_fftfin_fft); for M = 128 by a separable
// direct DFT at the 2n-1 x n lags it needs (k_fftfin).  A kernel boundary
// rather than a "last workgroup" handshake: the XCDs' L2 caches are not
// coherent, so a device-scope fence in every workgroup costs far more.
#include "rrc_device.h"
#include "rrc_launch.h"

namespace rrc {

// S samples per step; BOTH: one work-item computes both halves of a row,
// so the row is loaded and divided by the gains once
template <int M> struct FftCfg;
// NT: work-items of the M <= 64 kernel, a multiple of 2M (each half of a
// column transform spread over NT / (2M) work-items); M = 48 = 3 x 16 uses
// the radix-3 register FFT.
template <> struct FftCfg<16>  { static constexpr int S = 16; static constexpr bool BOTH = true; static constexpr int NT = 256; };
template <> struct FftCfg<32>  { static constexpr int S = 8; static constexpr bool BOTH = true; static constexpr int NT = 256; };
template <> struct FftCfg<48>  { static constexpr int S = 4; static constexpr bool BOTH = true; static constexpr int NT = 192; };
template <> struct FftCfg<64>  { static constexpr int S = 4; static constexpr bool BOTH = false; static constexpr int NT = 256; };
template <> struct FftCfg<96>  { static constexpr int S = 4; };   // k_fftcorr_t
template <> struct FftCfg<128> { static constexpr int S = 2; };   // k_fftcorr_q

constexpr int kFftThreads = 256;   // the finish kernels

template <int M>
constexpr int fft_samples_per_step() { return FftCfg<M>::S; }

// Loads voltage (y, k) of sample row `vrow` as a complex float.
template <bool CI4>
__device__ __forceinline__ float2 load_volt(const void* base, size_t idx);

template <>
__device__ __forceinline__ float2 load_volt<false>(const void* base, size_t idx) {
    return reinterpret_cast<const float2*>(base)[idx];
}
template <>
__device__ __forceinline__ float2 load_volt<true>(const void* base, size_t idx) {
    const int b = reinterpret_cast<const uint8_t*>(base)[idx];
    const int re = (b << 24) >> 28;            // sign-extended high nibble
    const int im = (b << 28) >> 28;            // sign-extended low nibble
    return make_float2((float)re, (float)im);
}

// Lag index of a canonical d in the V^unique layout.
__device__ __forceinline__ int lag_index(int n, int dx, int dy) {
    return dy == 0 ? dx - 1 : (n - 1) + (dy - 1) * (2 * n - 1) + (dx + n - 1);
}

// V(d) = C(d) / N_d (C already divided by M^2 T): N_d = (n - |dx|)(n - dy)
// on a full grid, else the masked lattice's table, and zero at a lag no
// pair of antennas realises.
__device__ __forceinline__ float2 lag_value(float2 c, int n, int dx, int dy, const float* __restrict__ ndt, int l) {
    const int adx = dx < 0 ? -dx : dx;
    const float nd = ndt ? ndt[l] : (float)((n - adx) * (n - dy));
    return nd > 0.0f ? make_float2(c.x / nd, c.y / nd) : make_float2(0.0f, 0.0f);
}

// Inverse transform of one unit's integrated power grid and redundant
// normalisation, by one workgroup, for M <= 64: C = conj(FFT2(P)) / M^2
// (P is real).  Only M/2-point FFTs are used, so the registers needed match
// the main loop.  Rows: P is real, so its M-point transform comes from one
// M/2-point FFT of z_k = P_{2k} + i P_{2k+1} (X_f = A_f + w^f B_f,
// X_{f+M/2} = A_f - w^f B_f with A, B the transforms of the even and odd
// samples, recovered from Z_f and conj(Z_{M/2-f})).  Columns: only
// dx in (-n, n) and dy in [0, n) are needed; two threads per column
// transform the even and odd rows, and X_dy = E_dy + w^dy O_dy.
// `lds` must hold M (M+1) + M^2 complex values.
// Sum of a unit's nchunk partial power grids, element by element in chunk
// order (deterministic).  Each work-item takes four consecutive grid points
// (16-byte loads) and keeps eight chunks' loads in flight at a time; the
// totals go to dst[row * RS + col].
template <int M, int NT, int RS>
__device__ __forceinline__ void sum_partials(const float* __restrict__ src, int nchunk, float* dst) {
    constexpr int Q4 = M * M / 4;
    const float4* s4 = reinterpret_cast<const float4*>(src);
    for (int q4 = threadIdx.x; q4 < Q4; q4 += NT) {
        float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
        int c = 0;
        for (; c + 8 <= nchunk; c += 8) {
            float4 v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = s4[(size_t)(c + u) * Q4 + q4];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                acc.x += v[u].x;
                acc.y += v[u].y;
                acc.z += v[u].z;
                acc.w += v[u].w;
            }
        }
        for (; c < nchunk; ++c) {
            const float4 v = s4[(size_t)c * Q4 + q4];
            acc.x += v.x;
            acc.y += v.y;
            acc.z += v.z;
            acc.w += v.w;
        }
        const int q = 4 * q4, row = q / M, col = q % M;
        float* d = dst + row * RS + col;
        d[0] = acc.x;
        d[1] = acc.y;
        d[2] = acc.z;
        d[3] = acc.w;
    }
}

template <int M>
__device__ __forceinline__ void inverse_to_lags(float2* lds, const float* __restrict__ src, int nchunk,
                                                int n, int T, float2* __restrict__ vunique,
                                                float* __restrict__ vauto, int unit,
                                                const float* __restrict__ ndt, int n_live) {
    constexpr int H = M / 2, RS = M + 1, NT = kFftThreads;
    float2* A = lds;                                       // [M][RS] row transforms
    float* psum = reinterpret_cast<float*>(lds + M * RS);  // [M][RS] integrated power
    float2* eo = lds + M * RS;                             // [2][M][H], reuses psum's space
    const int tid = threadIdx.x;
    sum_partials<M, NT, RS>(src, nchunk, psum);
    __syncthreads();
    if (tid < M) {
        float2 z[H];
#pragma unroll
        for (int k = 0; k < H; ++k) z[k] = make_float2(psum[tid * RS + 2 * k], psum[tid * RS + 2 * k + 1]);
        fft_dif<H>(z);
#pragma unroll
        for (int f = 0; f < H; ++f) {
            const float2 zf = z[index_of<H>(f)];
            const float2 zc = cconj(z[index_of<H>((H - f) % H)]);
            const float2 ev = make_float2(0.5f * (zf.x + zc.x), 0.5f * (zf.y + zc.y));
            const float2 od = make_float2(0.5f * (zf.y - zc.y), -0.5f * (zf.x - zc.x));
            const float2 wod = twmul<M>(od, f);
            A[tid * RS + f] = cadd(ev, wod);
            A[tid * RS + f + H] = csub(ev, wod);
        }
    }
    __syncthreads();
    {
        const int f = tid >> 1, h = tid & 1;
        const int dx = f < H ? f : f - M;
        if (tid < 2 * M && dx > -n && dx < n) {
            float2 x[H];
#pragma unroll
            for (int k = 0; k < H; ++k) x[k] = A[(2 * k + h) * RS + f];
            fft_dif<H>(x);
#pragma unroll
            for (int r = 0; r < H; ++r) eo[(h * M + f) * H + freq_of<H>(r)] = x[r];
        }
    }
    __syncthreads();
    const int nlag = 2 * n * (n - 1);
    const float norm = 1.0f / ((float)M * (float)M * (float)T);
    for (int q = tid; q < M * n; q += NT) {
        const int f = q / n, dy = q % n;
        const int dx = f < H ? f : f - M;
        if (dx <= -n || dx >= n || (dy == 0 && dx < 0)) continue;
        const float2 xv = cadd(eo[f * H + dy], twmul<M>(eo[(M + f) * H + dy], dy));
        const float2 c = make_float2(xv.x * norm, -xv.y * norm);
        if (dx == 0 && dy == 0) {
            vauto[unit] = c.x / (float)n_live;
        } else {
            const int l = lag_index(n, dx, dy);
            vunique[(size_t)unit * nlag + l] = lag_value(c, n, dx, dy, ndt, l);
        }
    }
}

// acc + |x|^2 as two chained FMAs (written as acc + (x.x x.x + x.y x.y) it
// compiles to a multiply, an FMA and an add)
__device__ __forceinline__ float acc_power(float acc, float2 x) {
    return fmaf(x.x, x.x, fmaf(x.y, x.y, acc));
}

// One half of a padded M-point transform whose upper M/2 inputs are zero:
// outputs 2r + ODD are the M/2-point transform of x, pre-twiddled by
// w_M^k for the odd ones.  Row stage: store them in natural order.
template <int M, bool ODD>
__device__ __forceinline__ void row_half(float2 (&x)[M / 2], float2* out) {
    constexpr int H = M / 2;
    if constexpr (ODD) {
#pragma unroll
        for (int k = 0; k < H; ++k) x[k] = twmul<M>(x[k], k);
    }
    fft_dif<H>(x);
#pragma unroll
    for (int r = 0; r < H; ++r) out[2 * freq_of<H>(r) + ODD] = x[r];
}

// Column stage: add the powers of the half's outputs (in bit-reversed
// order; the final reduction places them).
template <int M, bool ODD>
__device__ __forceinline__ void col_half(float2 (&x)[M / 2], float (&acc)[M / 2]) {
    constexpr int H = M / 2;
    if constexpr (ODD) {
#pragma unroll
        for (int k = 0; k < H; ++k) x[k] = twmul<M>(x[k], k);
    }
    fft_dif<H>(x);
#pragma unroll
    for (int r = 0; r < H; ++r) acc[r] = acc_power(acc[r], x[r]);
}

// W2: complex64 rows of even n, loaded as 16-byte pairs (half the load
// instructions; each lane reads its own row, so every load touches as many
// cache lines as there are lanes).
template <int M, bool CI4, bool W2 = false>
__global__ __launch_bounds__(FftCfg<M>::NT) void k_fftcorr(const void* __restrict__ volt,
                                                         const float2* __restrict__ gains,
                                                         float* __restrict__ ppart, int n, int T,
                                                         int tchunk, int nchunk,
                                                         const uint8_t* __restrict__ live) {
    constexpr int H = M / 2;
    constexpr int S = FftCfg<M>::S;
    constexpr int NT = FftCfg<M>::NT;
    constexpr int RS = M + 1;                     // padded LDS row stride (complex)
    constexpr bool BOTH = FftCfg<M>::BOTH;
    constexpr int CPT = 2 * M * S / NT;           // column tasks per thread (1 or 2)
    constexpr int G = S / CPT;                    // threads sharing one column half
    static_assert(G * M == NT / 2, "column tasks fill half the workgroup per half");
    static_assert(S * M / 2 <= (BOTH ? NT : NT / 2), "row tasks fit the workgroup");
    static_assert(CPT == 1 || CPT == 2, "column tasks per thread");
    static_assert(M * M <= 2 * S * H * RS, "power grid must fit in the row buffer");

    __shared__ float2 rbuf[S * H * RS];
    __shared__ float2 hinv[(H + 1) * (H + 1)];

    const int tid = threadIdx.x;
    const int unit = blockIdx.y;
    const int chunk = blockIdx.x;
    const int N = n * n;
    const int tb = chunk * tchunk;
    const int te = min(T, tb + tchunk);

    // 1/g on an (H+1) x (H+1) table, zero outside the n x n grid (and at
    // grid points of a masked lattice with no antenna): the padded inputs
    // of a row then come out zero without a branch per element, and row H
    // (all zero) serves the samples past the chunk end.
    for (int q = tid; q < (H + 1) * (H + 1); q += NT) {
        const int y = q / (H + 1), k = q % (H + 1);
        float2 h = make_float2(0.0f, 0.0f);
        if (y < n && k < n && (!live || live[y * n + k])) {
            const float2 g = gains[(size_t)unit * N + y * n + k];
            const float d = 1.0f / cabs2(g);
            h = make_float2(g.x * d, -g.y * d);
        }
        hinv[q] = h;
    }
    // rows n..H-1 of every sample's row buffer stay zero
    if (n < H) {
        for (int q = tid; q < S * (H - n) * RS; q += NT) {
            const int s = q / ((H - n) * RS), r = q % ((H - n) * RS);
            rbuf[(s * H + n) * RS + r] = make_float2(0.0f, 0.0f);
        }
    }

    float acc[H];
#pragma unroll
    for (int r = 0; r < H; ++r) acc[r] = 0.0f;

    // Row stage: with BOTH a work-item takes both halves of its row (one row
    // per work-item); otherwise the half (even / odd outputs) is uniform per
    // wave and only the waves of the odd half run the pre-twiddle.  Each
    // branch on a half runs through to the store (or, in the column stage,
    // the power sums), so the arrays of the two paths are never merged.
    const int rh = BOTH ? 0 : tid / (NT / 2);
    const int ry = BOTH ? tid % n : (tid % (NT / 2)) % n;
    const int rs = BOTH ? tid / n : (tid % (NT / 2)) / n;
    const bool row_active = rs < S;
    const int ch = tid / (NT / 2);
    const int cu = (tid % (NT / 2)) % M;
    const int cs0 = (tid % (NT / 2)) / M;

    __syncthreads();

    // complex64 rows of even n (16-byte pairs, H / 2 of them per row) are
    // loaded one step ahead at M = 64, so the loads are in flight during the
    // column stage (193 VGPRs, still the two waves per SIMD the LDS allows;
    // at M = 32 the extra registers would cost a wave per SIMD); a sample
    // past the chunk end re-reads the last one and meets the zero row of the
    // table, and columns k >= n re-read column n-2 and meet 1/g = 0
    constexpr bool PF = W2 && M == 64;
    float4 rq[PF ? H / 2 : 1];
    auto load_row = [&](int t0) {
        const int t = min(t0 + rs, te - 1);
        const float2* vr = reinterpret_cast<const float2*>(volt) + ((size_t)unit * T + t) * N + (size_t)ry * n;
#pragma unroll
        for (int k = 0; k < H; k += 2) rq[k / 2] = *reinterpret_cast<const float4*>(vr + min(k, n - 2));
    };
    if constexpr (PF) {
        if (row_active) load_row(tb);
    }

    for (int t0 = tb; t0 < te; t0 += S) {
        if (row_active) {
            float2 x[H];
            // a sample past the chunk end re-reads the last one and meets the
            // zero row of the table
            const bool live = t0 + rs < te;
            const int t = live ? t0 + rs : te - 1;
            const size_t rowbase = ((size_t)unit * T + t) * N + (size_t)ry * n;
            const float2* hrow = hinv + (live ? ry : H) * (H + 1);
            {
                // columns k >= n re-read column n-1 (finite) and meet 1/g = 0
                if constexpr (PF) {
#pragma unroll
                    for (int k = 0; k < H; k += 2) {
                        const float4 q = rq[k / 2];
                        x[k] = cmul(make_float2(q.x, q.y), hrow[k]);
                        x[k + 1] = cmul(make_float2(q.z, q.w), hrow[k + 1]);
                    }
                } else if constexpr (W2) {
                    const float2* vr = reinterpret_cast<const float2*>(volt) + rowbase;
#pragma unroll
                    for (int k = 0; k < H; k += 2) {
                        const float4 q = *reinterpret_cast<const float4*>(vr + min(k, n - 2));
                        x[k] = cmul(make_float2(q.x, q.y), hrow[k]);
                        x[k + 1] = cmul(make_float2(q.z, q.w), hrow[k + 1]);
                    }
                } else {
#pragma unroll
                    for (int k = 0; k < H; ++k)
                        x[k] = cmul(load_volt<CI4>(volt, rowbase + min(k, n - 1)), hrow[k]);
                }
            }
            float2* out = rbuf + (rs * H + ry) * RS;
            if constexpr (BOTH) {
                float2 y[H];
#pragma unroll
                for (int k = 0; k < H; ++k) y[k] = x[k];
                row_half<M, false>(x, out);
                row_half<M, true>(y, out);
            } else if (rh) {
                row_half<M, true>(x, out);
            } else {
                row_half<M, false>(x, out);
            }
        }
        __syncthreads();
        if constexpr (PF) {
            if (row_active && t0 + S < te) load_row(t0 + S);
        }
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
            const int s = cs0 + c * G;
            float2 x[H];
#pragma unroll
            for (int k = 0; k < H; ++k) x[k] = rbuf[(s * H + k) * RS + cu];
            if (ch)
                col_half<M, true>(x, acc);
            else
                col_half<M, false>(x, acc);
        }
        __syncthreads();
    }

    // Reduce the G partial grids that share a column half, in a fixed order.
    float* pl = reinterpret_cast<float*>(rbuf);
    for (int q = tid; q < M * M; q += NT) pl[q] = 0.0f;
    __syncthreads();
    for (int gidx = 0; gidx < G; ++gidx) {
        if (cs0 == gidx) {
#pragma unroll
            for (int r = 0; r < H; ++r) pl[(2 * freq_of<H>(r) + ch) * M + cu] += acc[r];
        }
        __syncthreads();
    }
    float* dst = ppart + ((size_t)unit * nchunk + chunk) * (M * M);
    for (int q = tid; q < M * M; q += NT) dst[q] = pl[q];
}


// ---------------------------------------------------------------- M = 128
// For 33 <= n <= 64 a whole M/2 = 64-point transform per work-item needs
// 128 registers of data plus 64 accumulators, and two samples' row buffers
// fill the LDS, so the M <= 64 kernel would run one wave per SIMD.  Here
// each transform is split by output residue mod 4 (a wave-uniform
// "quarter" q): with j' < 32,
//     E(4m + q) = sum_j' w_32^{j'm} w_128^{j'q} [x_j' + (-i)^q x_{j'+32}],
// a 32-point FFT after a fold of the 64 inputs.  512 work-items process two
// samples per step, one row or column per lane.  Row stage, in two halves:
// wave (s, R) loads input group R (eight pairs j, j + 32) of every row of
// sample s, divides by the gains and writes all four quarters' folded,
// twiddled inputs into that row of the row buffer; after a barrier wave
// (s, q) reads quarter q's 32 inputs back, transforms them and writes
// E(4m + q) over them, at column 32 q + m.  So every voltage is unpacked
// and divided by its gain once, not once per quarter, and a row's
// transform rewrites only the block its own lane read.  Column stage: wave
// (q, h) takes quarter q of the buffer's columns 64h .. 64h + 63 (natural
// columns 4 (c mod 32) + c div 32) of both samples, so each work-item owns
// 32 grid points of |E|^2 outright and writes them with no reduction.
//
// LDS: the two row buffers (128 KB) and the 1/g table (32 KB) fill the
// 160 KB, so nothing is padded.  The table is stored transposed ([k][y]),
// which makes the row stage's reads (lanes on rows) consecutive.  Row
// buffer entry (y, c) sits at column c ^ (y mod 32): row-stage writes
// (lanes on rows, one c) then spread over the banks, and column-stage
// reads (lanes on columns, one row) stay a permutation of consecutive
// words.  The XOR acts below bit 10 of the byte address, so every access
// is one XOR of a per-lane base with a constant plus an immediate offset.
constexpr int kQThreads = 512;

// W consecutive voltages from element idx (W divides n, so a group never
// straddles the end of a row): 4-bit as one 16- or 32-bit word, complex64
// as one 16-byte pair.
template <bool CI4, int W>
__device__ __forceinline__ void load_group(const void* base, size_t idx, float2 (&v)[W]) {
    if constexpr (CI4) {
        const uint8_t* b = reinterpret_cast<const uint8_t*>(base) + idx;
        uint32_t word;
        if constexpr (W == 4) word = *reinterpret_cast<const uint32_t*>(b);
        else if constexpr (W == 2) word = *reinterpret_cast<const uint16_t*>(b);
        else word = *b;
#pragma unroll
        for (int e = 0; e < W; ++e) {
            const int by = (int)((word >> (8 * e)) & 0xFFu);
            v[e] = make_float2((float)((by << 24) >> 28), (float)((by << 28) >> 28));
        }
    } else {
        const float2* f = reinterpret_cast<const float2*>(base) + idx;
        if constexpr (W == 2) {
            const float4 q = *reinterpret_cast<const float4*>(f);
            v[0] = make_float2(q.x, q.y);
            v[1] = make_float2(q.z, q.w);
        } else {
            v[0] = f[0];
        }
    }
}

__device__ __forceinline__ const float2& lds_at(const float2* lds, uint32_t byte_off) {
    return *reinterpret_cast<const float2*>(reinterpret_cast<const char*>(lds) + byte_off);
}

// Raw inputs of one row group (the eight pairs j, j + 32 with j in
// [8R, 8R + 8)): 4-bit as the loaded words (or half-words), complex64 as
// values.  Loaded one step ahead, so the loads are in flight during the
// column stage.
template <bool CI4, int W> struct RowRaw;
template <int W> struct RowRaw<true, W> { uint32_t w[16 / W]; };
template <int W> struct RowRaw<false, W> { float2 v[16]; };

// Two runs of eight inputs, from ja and from jb.  Inputs 32 .. 63 may lie
// past the row (n >= 33 keeps 0 .. 31 inside): their groups are clamped to
// the last one, and the 1/g table zeroes them.
template <bool CI4, int W>
__device__ __forceinline__ void row_load(const void* __restrict__ volt, size_t rowbase, int ja, int jb, int n,
                                         RowRaw<CI4, W>& raw) {
    const int nw = n - W;
#pragma unroll
    for (int e = 0; e < 8; e += W) {
        const size_t ia = rowbase + ja + e, ib = rowbase + min(jb + e, nw);
        if constexpr (CI4) {
            const uint8_t* b = reinterpret_cast<const uint8_t*>(volt);
            if constexpr (W == 4) {
                raw.w[e / W] = *reinterpret_cast<const uint32_t*>(b + ia);
                raw.w[8 / W + e / W] = *reinterpret_cast<const uint32_t*>(b + ib);
            } else {
                static_assert(W == 2, "4-bit groups of two or four");
                raw.w[e / W] = *reinterpret_cast<const uint16_t*>(b + ia);
                raw.w[8 / W + e / W] = *reinterpret_cast<const uint16_t*>(b + ib);
            }
        } else {
            float2 ga[W], gb[W];
            load_group<false, W>(volt, ia, ga);
            load_group<false, W>(volt, ib, gb);
#pragma unroll
            for (int f = 0; f < W; ++f) {
                raw.v[e + f] = ga[f];
                raw.v[8 + e + f] = gb[f];
            }
        }
    }
}

// Row stage, first half: group R of one row.  x = v / g for both inputs of
// each pair, then every quarter's folded, twiddled input
// u_q(j) = w_128^{jq} [x_j + (-i)^q x_{j+32}] goes to the row's own LDS row
// at column 32 q + j (swizzled).  Each input is divided by its gain once;
// the quarter waves that transform the row read u_q back.
// hcol = table + y; wbase = byte offset of the row | (y mod 32) << 3.
template <int R, bool CI4, int W>
__device__ __forceinline__ void row_fold(const RowRaw<CI4, W>& raw, const float2* hcol, float2* rbuf,
                                         uint32_t wbase) {
    float2 a[8], b[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        if constexpr (CI4) {
            const int wa = (int)((raw.w[e / W] >> (8 * (e % W))) & 0xFFu);
            const int wb = (int)((raw.w[8 / W + e / W] >> (8 * (e % W))) & 0xFFu);
            a[e] = make_float2((float)((wa << 24) >> 28), (float)((wa << 28) >> 28));
            b[e] = make_float2((float)((wb << 24) >> 28), (float)((wb << 28) >> 28));
        } else {
            a[e] = raw.v[e];
            b[e] = raw.v[8 + e];
        }
    }
    char* rb = reinterpret_cast<char*>(rbuf);
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int j = 8 * R + e;
        const float2 xa = cmul(a[e], hcol[j * 64]);
        const float2 xb = cmul(b[e], hcol[(j + 32) * 64]);
#pragma unroll
        for (int q = 0; q < 4; ++q)
            *reinterpret_cast<float2*>(rb + (wbase ^ ((32 * q + j) << 3))) =
                twmul<128>(cadd(xa, twmul<4>(xb, q)), j * q);
    }
}

// Row stage, second half: quarter Q of one row, the 32-point transform of
// u_Q read back from the row, its outputs E(4m + Q) written over u_Q: output
// m goes to column 32 Q + m, the block u_Q occupied, so each lane rewrites
// only what it has read and no other wave needs to have read first.
template <int Q>
__device__ __forceinline__ void row_transform(float2* rbuf, uint32_t wbase) {
    float2 u[32];
#pragma unroll
    for (int j = 0; j < 32; ++j) u[j] = lds_at(rbuf, wbase ^ ((32 * Q + j) << 3));
    fft_dif<32>(u);
    char* rb = reinterpret_cast<char*>(rbuf);
#pragma unroll
    for (int r = 0; r < 32; ++r)
        *reinterpret_cast<float2*>(rb + (wbase ^ ((32 * Q + bitrev<32>(r)) << 3))) = u[r];
}

// Quarter Q of one column of one sample's row buffer; |E|^2 into acc.
// rbase = byte offset of the sample's buffer | u << 3.
template <int Q>
__device__ __forceinline__ void col_quarter(const float2* rbuf, uint32_t rbase, float (&acc)[32]) {
    float2 v[32];
#pragma unroll
    for (int j = 0; j < 32; ++j) {
        const uint32_t o = rbase ^ (j << 3);
        const float2 a = lds_at(rbuf, o + j * 1024);
        const float2 b = lds_at(rbuf, o + (j + 32) * 1024);
        v[j] = twmul<128>(cadd(a, twmul<4>(b, Q)), j * Q);
    }
    fft_dif<32>(v);
#pragma unroll
    for (int r = 0; r < 32; ++r) acc[r] = acc_power(acc[r], v[r]);
}

template <bool CI4, int W>
__global__ __launch_bounds__(kQThreads) void k_fftcorr_q(const void* __restrict__ volt,
                                                         const float2* __restrict__ gains,
                                                         float* __restrict__ ppart, int n, int T,
                                                         int tchunk, int nchunk,
                                                         const uint8_t* __restrict__ live) {
    constexpr int M = 128, H = 64, S = FftCfg<128>::S, NT = kQThreads;
    static_assert(NT == 4 * 64 * S, "one row quarter per wave and sample");
    static_assert(M * 8 == 1024, "row stride of 1 KiB: the swizzle stays below bit 10");
    // (the launcher guarantees 33 <= n <= 64)
    __shared__ float2 rbuf[S * H * M];   // [s][y][c ^ (y mod 32)]
    __shared__ float2 hinv[H * H];       // [k][y], zero outside the grid

    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int unit = blockIdx.y;
    const int chunk = blockIdx.x;
    const int N = n * n;
    const int tb = chunk * tchunk;
    const int te = min(T, tb + tchunk);

    for (int q = tid; q < H * H; q += NT) {
        const int k = q / H, y = q % H;
        float2 h = make_float2(0.0f, 0.0f);
        if (y < n && k < n && (!live || live[y * n + k])) {
            const float2 g = gains[(size_t)unit * N + y * n + k];
            const float d = 1.0f / cabs2(g);
            h = make_float2(g.x * d, -g.y * d);
        }
        hinv[q] = h;
    }
    // rows n .. H-1 of both sample buffers stay zero
    for (int q = tid; q < S * (H - n) * M; q += NT) {
        const int s = q / ((H - n) * M), r = q % ((H - n) * M);
        rbuf[(s * H + n) * M + r] = make_float2(0.0f, 0.0f);
    }

    float acc[32];
#pragma unroll
    for (int r = 0; r < 32; ++r) acc[r] = 0.0f;
    const int rs = wave >> 2, rq = wave & 3;                 // row stage: sample, quarter
    const int cq = wave >> 1, cu = (wave & 1) * 64 + lane;   // column stage
    const int y = lane;
    __syncthreads();

    // 4-bit inputs (four or eight registers) are loaded one step ahead;
    // complex64 ones (32 registers) would spill, so they are loaded in step
    constexpr bool PF = CI4;
    RowRaw<CI4, W> raw;
    auto rowbase_of = [&](int t) { return ((size_t)unit * T + t) * N + (size_t)y * n; };
    if (PF && tb + rs < te && y < n) row_load<CI4, W>(volt, rowbase_of(tb + rs), 8 * rq, 8 * rq + 32, n, raw);
    for (int t0 = tb; t0 < te; t0 += S) {
        const int t = t0 + rs;
        const bool row_lane = t < te && y < n;
        // byte offset of row y of sample rs | (y mod 32) << 3, recomputed per
        // step so the swizzled addresses are not hoisted into registers for
        // the whole loop
        uint32_t wbase = (uint32_t)((rs * H + y) * M * 8) | (uint32_t)((y & 31) << 3);
        asm volatile("" : "+v"(wbase));
        if (row_lane) {
            if constexpr (!PF) row_load<CI4, W>(volt, rowbase_of(t), 8 * rq, 8 * rq + 32, n, raw);
            switch (rq) {
                case 0: row_fold<0, CI4, W>(raw, hinv + y, rbuf, wbase); break;
                case 1: row_fold<1, CI4, W>(raw, hinv + y, rbuf, wbase); break;
                case 2: row_fold<2, CI4, W>(raw, hinv + y, rbuf, wbase); break;
                default: row_fold<3, CI4, W>(raw, hinv + y, rbuf, wbase); break;
            }
        }
        __syncthreads();
        if (row_lane) {
            switch (rq) {
                case 0: row_transform<0>(rbuf, wbase); break;
                case 1: row_transform<1>(rbuf, wbase); break;
                case 2: row_transform<2>(rbuf, wbase); break;
                default: row_transform<3>(rbuf, wbase); break;
            }
        }
        __syncthreads();
        // the next step's inputs, in flight during the column stage
        if (PF && t + S < te && y < n) row_load<CI4, W>(volt, rowbase_of(t + S), 8 * rq, 8 * rq + 32, n, raw);
        const int ns = min(S, te - t0);
        for (int s = 0; s < ns; ++s) {
            uint32_t rbase = (uint32_t)(s * H * M * 8) | (uint32_t)(cu << 3);
            asm volatile("" : "+v"(rbase));
            switch (cq) {
                case 0: col_quarter<0>(rbuf, rbase, acc); break;
                case 1: col_quarter<1>(rbuf, rbase, acc); break;
                case 2: col_quarter<2>(rbuf, rbase, acc); break;
                default: col_quarter<3>(rbuf, rbase, acc); break;
            }
        }
        __syncthreads();
    }

    // grid point (ky, kx) = (4 bitrev(r) + cq, kx), where the row buffer's
    // column cu = 32 q' + m holds kx = 4 m + q'
    const int kx = 4 * (cu & 31) + (cu >> 5);
    float* dst = ppart + ((size_t)unit * nchunk + chunk) * (M * M);
#pragma unroll
    for (int r = 0; r < 32; ++r) dst[(4 * bitrev<32>(r) + cq) * M + kx] = acc[r];
}

// ------------------------------------------------------------------ M = 96
// Grids of 33 .. 48 points per side need 2n - 1 <= 95 points of padded
// transform, so 96 serves where 128 would pad 1.78x more grid points.
// With x_j = 0 for j >= 48, E(3m + q) = sum_j w_32^{mj} u_q(j) for
// u_q(j) = w_96^{qj} [x_j + w_3^q x_{j+32}]: three 32-point transforms (the
// thirds q) per row and per column, the 96-point analogue of the quarter
// split above.  Nine waves, three per third, four samples per step.
//  - Row stage: the 192 lanes of third q's waves take (sample, row) =
//    (i / 48, i % 48); row group q holds inputs j in [8q, 8q + 8) with their
//    partners j + 32 (q = 0, 1), or j in [16, 32) (q = 2).  Each input is
//    divided by its gain once, every third's u(j) written to the row.
//  - Column stage: lanes take (p, c) = (i / 96, i % 96), samples p and
//    p + 2 of the step, column c; the two lanes of one (q, c) add their
//    sums at the end.
// Row buffer: rows r = 48 s + y of 96 complex (768 B); entry (r, c) sits at
// column 32 (c / 32) + ((c mod 32) ^ (r mod 32)).  The four samples' rows
// take 144 KiB of LDS, so the 1/g table comes from the workspace (18 KiB
// per unit, L1-resident) instead of LDS.
constexpr int kTThreads = 576;
constexpr int kTFrame = 48;           // the 1/g table's frame: [k][y], k, y < 48

// 1/g of every antenna, [U][k][y] on the 48 x 48 frame, zero outside the
// grid and at dead grid points.
__global__ __launch_bounds__(256) void k_hinv48(const float2* __restrict__ gains, float2* __restrict__ hinv,
                                                int n, const uint8_t* __restrict__ live) {
    constexpr int F = kTFrame;
    const int unit = blockIdx.x;
    const int N = n * n;
    for (int x = threadIdx.x; x < F * F; x += 256) {
        const int k = x / F, y = x % F;
        float2 h = make_float2(0.0f, 0.0f);
        if (y < n && k < n && (!live || live[y * n + k])) {
            const float2 g = gains[(size_t)unit * N + y * n + k];
            const float d = 1.0f / cabs2(g);
            h = make_float2(g.x * d, -g.y * d);
        }
        hinv[(size_t)unit * (F * F) + x] = h;
    }
}

// Row stage, first half, third kernel: row group R (see above); hrow =
// the unit's 1/g table + y; wbase = byte offset of the row | (r mod 32) << 3.
template <int R, bool CI4, int W>
__device__ __forceinline__ void row_fold_t(const RowRaw<CI4, W>& raw, const float2* __restrict__ hrow,
                                           float2* rbuf, uint32_t wbase) {
    float2 a[8], b[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        if constexpr (CI4) {
            const int wa = (int)((raw.w[e / W] >> (8 * (e % W))) & 0xFFu);
            const int wb = (int)((raw.w[8 / W + e / W] >> (8 * (e % W))) & 0xFFu);
            a[e] = make_float2((float)((wa << 24) >> 28), (float)((wa << 28) >> 28));
            b[e] = make_float2((float)((wb << 24) >> 28), (float)((wb << 28) >> 28));
        } else {
            a[e] = raw.v[e];
            b[e] = raw.v[8 + e];
        }
    }
    char* rb = reinterpret_cast<char*>(rbuf);
    if constexpr (R < 2) {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const int j = 8 * R + e;
            const float2 xa = cmul(a[e], hrow[j * kTFrame]);
            const float2 xb = cmul(b[e], hrow[(j + 32) * kTFrame]);
#pragma unroll
            for (int q = 0; q < 3; ++q)
                *reinterpret_cast<float2*>(rb + (wbase ^ (j << 3)) + 256 * q) =
                    twmul<96>(cadd(xa, twmul<96>(xb, 32 * q)), j * q);
        }
    } else {
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int j = 16 + e;
            const float2 x = cmul(e < 8 ? a[e] : b[e - 8], hrow[j * kTFrame]);
#pragma unroll
            for (int q = 0; q < 3; ++q)
                *reinterpret_cast<float2*>(rb + (wbase ^ (j << 3)) + 256 * q) = twmul<96>(x, j * q);
        }
    }
}

// Row stage, second half: third Q of one row, its outputs E(3m + Q) written
// over its inputs (output m at column 32 Q + m).
template <int Q>
__device__ __forceinline__ void row_transform_t(float2* rbuf, uint32_t wbase) {
    float2 u[32];
#pragma unroll
    for (int j = 0; j < 32; ++j) u[j] = lds_at(rbuf, (wbase ^ (j << 3)) + 256 * Q);
    fft_dif<32>(u);
    char* rb = reinterpret_cast<char*>(rbuf);
#pragma unroll
    for (int r = 0; r < 32; ++r)
        *reinterpret_cast<float2*>(rb + (wbase ^ (bitrev<32>(r) << 3)) + 256 * Q) = u[r];
}

// Third Q of one column of one sample's rows; |E|^2 into acc.  rbase =
// byte offset of the sample's rows + 256 (c / 32) | ((c mod 32) ^ 16 (s mod 2))
// << 3: row j's entry is then (rbase ^ (j << 3)) + 768 j, and row j + 32
// shares row j's swizzle.
template <int Q>
__device__ __forceinline__ void col_third(const float2* rbuf, uint32_t rbase, float (&acc)[32]) {
    float2 v[32];
#pragma unroll
    for (int j = 0; j < 32; ++j) {
        const uint32_t o = rbase ^ (j << 3);
        const float2 a = lds_at(rbuf, o + j * 768);
        if (j < 16) {
            const float2 b = lds_at(rbuf, o + (j + 32) * 768);
            v[j] = twmul<96>(cadd(a, twmul<96>(b, 32 * Q)), j * Q);
        } else {
            v[j] = twmul<96>(a, j * Q);
        }
    }
    fft_dif<32>(v);
#pragma unroll
    for (int r = 0; r < 32; ++r) acc[r] = acc_power(acc[r], v[r]);
}

template <bool CI4, int W>
__global__ __launch_bounds__(kTThreads) void k_fftcorr_t(const void* __restrict__ volt,
                                                         const float2* __restrict__ hinv,
                                                         float* __restrict__ ppart, int n, int T,
                                                         int tchunk, int nchunk) {
    constexpr int M = 96, H = 48, S = FftCfg<96>::S, NT = kTThreads;
    constexpr int RB = H * M * 8;                 // bytes of one sample's rows
    static_assert(NT == 9 * 64 && S * H == 3 * 64, "three waves per third: four samples of 48 rows");
    static_assert(RB % 256 == 0, "the swizzle stays below bit 8");
    // (the launcher guarantees 33 <= n <= 48)
    __shared__ float2 rbuf[S * H * M];

    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int q = wave / 3;
    const int i = (wave - 3 * q) * 64 + (tid & 63);
    const int unit = blockIdx.y;
    const int chunk = blockIdx.x;
    const int N = n * n;
    const int tb = chunk * tchunk;
    const int te = min(T, tb + tchunk);

    // rows n .. 47 of every sample stay zero
    for (int x = tid; x < S * (H - n) * M; x += NT) {
        const int s = x / ((H - n) * M), r = x % ((H - n) * M);
        rbuf[(s * H + n) * M + r] = make_float2(0.0f, 0.0f);
    }

    float acc[32];
#pragma unroll
    for (int r = 0; r < 32; ++r) acc[r] = 0.0f;
    const int rs = i / H, y = i - H * rs;          // row stage: sample, row (row i of the buffer)
    const int cp = i / M, cc = i - M * cp;         // column stage: sample parity, column
    const int ja = q < 2 ? 8 * q : 16, jb = q < 2 ? 8 * q + 32 : 24;
    const float2* hunit = hinv + (size_t)unit * (kTFrame * kTFrame);
    __syncthreads();

    constexpr bool PF = CI4;
    RowRaw<CI4, W> raw;
    auto rowbase_of = [&](int t) { return ((size_t)unit * T + t) * N + (size_t)y * n; };
    if (PF && tb + rs < te && y < n) row_load<CI4, W>(volt, rowbase_of(tb + rs), ja, jb, n, raw);
    for (int t0 = tb; t0 < te; t0 += S) {
        const int t = t0 + rs;
        const bool row_lane = t < te && y < n;
        uint32_t wbase = (uint32_t)(i * M * 8) | (uint32_t)((i & 31) << 3);
        asm volatile("" : "+v"(wbase));
        // the 16 1/g values are re-read each step (from L1), not held in
        // registers across the loop
        int hoff = y;
        asm volatile("" : "+v"(hoff));
        const float2* hrow = hunit + hoff;
        if (row_lane) {
            if constexpr (!PF) row_load<CI4, W>(volt, rowbase_of(t), ja, jb, n, raw);
            switch (q) {
                case 0: row_fold_t<0, CI4, W>(raw, hrow, rbuf, wbase); break;
                case 1: row_fold_t<1, CI4, W>(raw, hrow, rbuf, wbase); break;
                default: row_fold_t<2, CI4, W>(raw, hrow, rbuf, wbase); break;
            }
        }
        __syncthreads();
        if (row_lane) {
            switch (q) {
                case 0: row_transform_t<0>(rbuf, wbase); break;
                case 1: row_transform_t<1>(rbuf, wbase); break;
                default: row_transform_t<2>(rbuf, wbase); break;
            }
        }
        __syncthreads();
        // the next step's inputs, in flight during the column stage
        if (PF && t + S < te && y < n) row_load<CI4, W>(volt, rowbase_of(t + S), ja, jb, n, raw);
        const int ns = min(S, te - t0);
        uint32_t rbase = (uint32_t)(cp * RB + 256 * (cc >> 5)) | (uint32_t)(((cc & 31) ^ (16 * cp)) << 3);
        asm volatile("" : "+v"(rbase));
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            if (cp + 2 * k < ns) {
                switch (q) {
                    case 0: col_third<0>(rbuf, rbase + k * 2 * RB, acc); break;
                    case 1: col_third<1>(rbuf, rbase + k * 2 * RB, acc); break;
                    default: col_third<2>(rbuf, rbase + k * 2 * RB, acc); break;
                }
            }
        }
        __syncthreads();
    }

    // the lanes of odd samples hand their sums to the even ones' lanes
    // through LDS ([q][r][c]), which add them in a fixed order; grid point
    // (ky, kx) = (3 bitrev(r) + q, kx), where column cc = 32 q' + m holds
    // kx = 3 m + q'
    float* red = reinterpret_cast<float*>(rbuf);
    if (cp == 1) {
#pragma unroll
        for (int r = 0; r < 32; ++r) red[(q * 32 + r) * M + cc] = acc[r];
    }
    __syncthreads();
    if (cp == 0) {
        const int kx = 3 * (cc & 31) + (cc >> 5);
        float* dst = ppart + ((size_t)unit * nchunk + chunk) * (M * M);
#pragma unroll
        for (int r = 0; r < 32; ++r) dst[(3 * bitrev<32>(r) + q) * M + kx] = acc[r] + red[(q * 32 + r) * M + cc];
    }
}

constexpr int kFinThreads = 256;
// lags dx per pass of the direct finish: at M = 128 a block of 8 keeps the
// workgroup's LDS (the M x M power grid plus M x DB partial sums) under
// half a CU, so two units share one
template <int M>
constexpr int fin_dx_block() { return M == 128 ? 8 : 32; }

template <int M>
__global__ __launch_bounds__(kFinThreads) void k_fftfin(const float* __restrict__ ppart, int nchunk,
                                                        int n, int T, float2* __restrict__ vunique,
                                                        float* __restrict__ vauto,
                                                        unsigned long long* __restrict__ stamps,
                                                        const float* __restrict__ ndt, int n_live) {
    constexpr int NT = kFinThreads;
    constexpr int DB = fin_dx_block<M>();
    __shared__ float pw[M * M];
    __shared__ float2 twp[M];              // e^{+2 pi i k / M}
    __shared__ float2 abuf[M * DB];

    const int tid = threadIdx.x;
    const int unit = blockIdx.x;
    const int nlag = 2 * n * (n - 1);
    const float* src = ppart + (size_t)unit * nchunk * (M * M);
    sum_partials<M, NT, M>(src, nchunk, pw);
    for (int k = tid; k < M; k += NT) twp[k] = make_float2(Tw<M>::t.re[k], -Tw<M>::t.im[k]);
    __syncthreads();

    const float norm = 1.0f / ((float)M * (float)M * (float)T);
    for (int dx0 = -(n - 1); dx0 <= n - 1; dx0 += DB) {
        // stage x: A(u_y, dx) = sum_{u_x} P(u_y, u_x) e^{+2 pi i u_x dx / M}
        for (int q = tid; q < M * DB; q += NT) {
            const int uy = q / DB, di = q % DB;
            const int dx = dx0 + di;
            float2 a = make_float2(0.0f, 0.0f);
            if (dx <= n - 1) {
                const float* prow = pw + uy * M;
                if constexpr ((M & (M - 1)) == 0) {
                    for (int ux = 0; ux < M; ++ux) {
                        const float2 w = twp[(ux * dx) & (M - 1)];
                        a.x += prow[ux] * w.x;
                        a.y += prow[ux] * w.y;
                    }
                } else {
                    const int step = dx < 0 ? dx + M : dx;     // ux dx mod M, stepped
                    int k = 0;
                    for (int ux = 0; ux < M; ++ux) {
                        const float2 w = twp[k];
                        a.x += prow[ux] * w.x;
                        a.y += prow[ux] * w.y;
                        k += step;
                        if (k >= M) k -= M;
                    }
                }
            }
            abuf[q] = a;
        }
        __syncthreads();
        // stage y: C(dx, dy) = sum_{u_y} A(u_y, dx) e^{+2 pi i u_y dy / M}
        for (int q = tid; q < n * DB; q += NT) {
            const int dy = q / DB, di = q % DB;
            const int dx = dx0 + di;
            if (dx > n - 1 || (dy == 0 && dx < 0)) continue;
            float2 c = make_float2(0.0f, 0.0f);
            if constexpr ((M & (M - 1)) == 0) {
                for (int uy = 0; uy < M; ++uy) c = cadd(c, cmul(abuf[uy * DB + di], twp[(uy * dy) & (M - 1)]));
            } else {
                int k = 0;
                for (int uy = 0; uy < M; ++uy) {
                    c = cadd(c, cmul(abuf[uy * DB + di], twp[k]));
                    k += dy;
                    if (k >= M) k -= M;
                }
            }
            if (dx == 0 && dy == 0) {
                vauto[unit] = c.x * norm / (float)n_live;
            } else {
                const int l = lag_index(n, dx, dy);
                vunique[(size_t)unit * nlag + l] = lag_value(make_float2(c.x * norm, c.y * norm), n, dx, dy, ndt, l);
            }
        }
        __syncthreads();
    }
    if (stamps && tid == 0) unit_done_stamp(stamps, unit);   // after the loop's last barrier
}

// Finish for M <= 64: one workgroup per unit, register FFTs (see
// inverse_to_lags).
template <int M>
__global__ __launch_bounds__(kFftThreads) void k_fftfin_fft(const float* __restrict__ ppart, int nchunk,
                                                            int n, int T, float2* __restrict__ vunique,
                                                            float* __restrict__ vauto,
                                                            unsigned long long* __restrict__ stamps,
                                                            const float* __restrict__ ndt, int n_live) {
    __shared__ float2 lds[M * (M + 1) + M * M];
    const int unit = blockIdx.x;
    inverse_to_lags<M>(lds, ppart + (size_t)unit * nchunk * (M * M), nchunk, n, T, vunique, vauto, unit, ndt,
                       n_live);
    if (stamps) {
        __syncthreads();
        if (threadIdx.x == 0) unit_done_stamp(stamps, unit);
    }
}

template <bool CI4, int W>
static void launch_q(const FftLaunch& L, hipStream_t st) {
    hipLaunchKernelGGL((k_fftcorr_q<CI4, W>), dim3(L.nchunk, L.n_units), dim3(kQThreads), 0, st, L.volt,
                       L.gains, L.ppart, L.n, L.T, L.tchunk, L.nchunk, L.mt.live);
}

template <bool CI4, int W>
static void launch_t(const FftLaunch& L, hipStream_t st) {
    hipLaunchKernelGGL((k_fftcorr_t<CI4, W>), dim3(L.nchunk, L.n_units), dim3(kTThreads), 0, st, L.volt,
                       L.hinv, L.ppart, L.n, L.T, L.tchunk, L.nchunk);
}

template <int M, bool CI4>
static hipError_t launch_fft_m(const FftLaunch& L, hipStream_t st) {
    if constexpr (M == 96) {
        if (L.n < 33 || L.n > 48 || (CI4 && (L.n & 1)) || !L.hinv) return hipErrorInvalidValue;
        hipLaunchKernelGGL(k_hinv48, dim3(L.n_units), dim3(256), 0, st, L.gains, L.hinv, L.n, L.mt.live);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        if constexpr (CI4) {
            if (L.n % 4 == 0) launch_t<true, 4>(L, st);
            else launch_t<true, 2>(L, st);
        } else {
            if (L.n % 2 == 0) launch_t<false, 2>(L, st);
            else launch_t<false, 1>(L, st);
        }
    } else if constexpr (M == 128) {
        // widest load group that divides n (4-bit plans have n even)
        if (L.n < 33 || L.n > 64 || (CI4 && (L.n & 1))) return hipErrorInvalidValue;
        if constexpr (CI4) {
            if (L.n % 4 == 0) launch_q<true, 4>(L, st);
            else launch_q<true, 2>(L, st);
        } else {
            if (L.n % 2 == 0) launch_q<false, 2>(L, st);
            else launch_q<false, 1>(L, st);
        }
    } else {
        dim3 grid1(L.nchunk, L.n_units);
        if (!CI4 && L.n % 2 == 0)
            hipLaunchKernelGGL((k_fftcorr<M, CI4, !CI4>), grid1, dim3(FftCfg<M>::NT), 0, st, L.volt, L.gains,
                               L.ppart, L.n, L.T, L.tchunk, L.nchunk, L.mt.live);
        else
            hipLaunchKernelGGL((k_fftcorr<M, CI4, false>), grid1, dim3(FftCfg<M>::NT), 0, st, L.volt, L.gains,
                               L.ppart, L.n, L.T, L.tchunk, L.nchunk, L.mt.live);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if constexpr (M <= 64) {
        hipLaunchKernelGGL((k_fftfin_fft<M>), dim3(L.n_units), dim3(kFftThreads), 0, st, L.ppart,
                           L.nchunk, L.n, L.T, L.vunique, L.vauto, L.stamps, L.mt.nd, L.mt.n_live);
    } else {
        hipLaunchKernelGGL((k_fftfin<M>), dim3(L.n_units), dim3(kFinThreads), 0, st, L.ppart,
                           L.nchunk, L.n, L.T, L.vunique, L.vauto, L.stamps, L.mt.nd, L.mt.n_live);
    }
    return hipGetLastError();
}

int fft_samples_per_step_for(int M) {
    switch (M) {
        case 16: return fft_samples_per_step<16>();
        case 32: return fft_samples_per_step<32>();
        case 48: return fft_samples_per_step<48>();
        case 64: return fft_samples_per_step<64>();
        case 96: return fft_samples_per_step<96>();
        case 128: return fft_samples_per_step<128>();
        default: return 0;
    }
}

hipError_t launch_fftcorr(const FftLaunch& L, hipStream_t st) {
    switch (L.M) {
        case 16: return L.ci4 ? launch_fft_m<16, true>(L, st) : launch_fft_m<16, false>(L, st);
        case 32: return L.ci4 ? launch_fft_m<32, true>(L, st) : launch_fft_m<32, false>(L, st);
        case 48: return L.ci4 ? launch_fft_m<48, true>(L, st) : launch_fft_m<48, false>(L, st);
        case 64: return L.ci4 ? launch_fft_m<64, true>(L, st) : launch_fft_m<64, false>(L, st);
        case 96: return L.ci4 ? launch_fft_m<96, true>(L, st) : launch_fft_m<96, false>(L, st);
        case 128: return L.ci4 ? launch_fft_m<128, true>(L, st) : launch_fft_m<128, false>(L, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace rrc
