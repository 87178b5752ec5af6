// Device-side helpers shared by the HIP kernels: complex arithmetic,
// compile-time twiddles, an in-register radix-2^2 FFT, and the implicit
// geometry of a square grid with a list of selected baseline-types.
#pragma once

#ifdef RRC_HOST_EMU
#include "rrc_emu.h"   // CPU build of the kernels' bodies, for host-side tests
#else
#include <hip/hip_runtime.h>
#endif
#include <stdint.h>

#define RRC_HD __host__ __device__ __forceinline__

namespace rrc {

constexpr int kMaxTypes = 16;

// ------------------------------------------------------------------ complex

RRC_HD float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
RRC_HD float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
RRC_HD float2 cmul(float2 a, float2 b) { return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
// a * conj(b)
RRC_HD float2 cmulc(float2 a, float2 b) { return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y); }
RRC_HD float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
RRC_HD float cabs2(float2 a) { return a.x * a.x + a.y * a.y; }

RRC_HD double2 dadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
RRC_HD double2 dsub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
RRC_HD double2 dmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
RRC_HD double2 dmulc(double2 a, double2 b) { return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y); }
RRC_HD double2 dconj(double2 a) { return make_double2(a.x, -a.y); }
RRC_HD double dabs2(double2 a) { return a.x * a.x + a.y * a.y; }
RRC_HD double2 to_d(float2 a) { return make_double2(a.x, a.y); }
RRC_HD float2 to_f(double2 a) { return make_float2((float)a.x, (float)a.y); }

// ------------------------------------------------- compile-time twiddles
//
// e^{-2 pi i k / L} evaluated in double at compile time.  The angle is
// reduced to an octant, so multiples of pi/4 come out exact (0, +-1,
// +-sqrt(1/2)) and the remaining values are Taylor series on [0, pi/4].

constexpr double kPi = 3.14159265358979323846;

constexpr double cx_sin(double x) {
    double x2 = x * x, term = x, sum = x;
    for (int i = 1; i < 14; ++i) { term *= -x2 / ((2.0 * i) * (2.0 * i + 1.0)); sum += term; }
    return sum;
}
constexpr double cx_cos(double x) {
    double x2 = x * x, term = 1.0, sum = 1.0;
    for (int i = 1; i < 14; ++i) { term *= -x2 / ((2.0 * i - 1.0) * (2.0 * i)); sum += term; }
    return sum;
}

struct cd { double re, im; };

// (cos t, sin t) for t = 2 pi k / L, k in [0, L)
constexpr cd cx_cis(int k, int L) {
    k %= L;
    if (k < 0) k += L;
    const long q = 8L * k;
    const int o = (int)(q / L);
    const long rem = q - (long)o * L;
    const double psi = (kPi / 4.0) * ((double)rem / (double)L);
    const double phi = (kPi / 4.0) * ((double)(L - rem) / (double)L);
    const double cp = cx_cos(psi), sp = cx_sin(psi);
    const double cf = cx_cos(phi), sf = cx_sin(phi);
    switch (o) {
        case 0: return cd{cp, sp};
        case 1: return cd{sf, cf};
        case 2: return cd{-sp, cp};
        case 3: return cd{-cf, sf};
        case 4: return cd{-cp, -sp};
        case 5: return cd{-sf, -cf};
        case 6: return cd{sp, -cp};
        default: return cd{cf, -sf};
    }
}

template <int L>
struct TwTable {
    float re[L];
    float im[L];   // e^{-2 pi i k / L} = re + i im
    constexpr TwTable() : re(), im() {
        for (int k = 0; k < L; ++k) {
            cd c = cx_cis(k, L);
            re[k] = (float)c.re;
            im[k] = (float)(-c.im);
        }
    }
};

template <int L>
struct Tw {
    static constexpr TwTable<L> t{};
};

// d * e^{-2 pi i k / L}; k is a compile-time constant after unrolling, so
// the trivial factors reduce to swaps and sign flips.
template <int L>
RRC_HD float2 twmul(float2 d, int k) {
    if (k == 0) return d;
    if (4 * k == L) return make_float2(d.y, -d.x);
    if (2 * k == L) return make_float2(-d.x, -d.y);
    if (4 * k == 3 * L) return make_float2(-d.y, d.x);
    constexpr float s = 0.70710678118654752440f;
    if (8 * k == L) return make_float2((d.x + d.y) * s, (d.y - d.x) * s);
    if (8 * k == 3 * L) return make_float2((d.y - d.x) * s, -(d.x + d.y) * s);
    const float c = Tw<L>::t.re[k], sn = Tw<L>::t.im[k];
    return make_float2(d.x * c - d.y * sn, d.x * sn + d.y * c);
}

// In-register decimation-in-frequency FFT of length L (a power of two):
// X[f] = sum_k x[k] e^{-2 pi i f k / L}, natural-order input, output
// element r holds frequency bitrev(r).
//
// The radix-2 stages are taken two at a time (radix 2^2).  In a block of
// 2h elements, the first stage's twiddle on element j + h/2 is w_2h^j
// times w_2h^{h/2} = -i, so the -i is applied inside the butterfly and
// w_2h^j moves past the second stage; the four outputs of (j, j + h/2,
// j + h, j + 3h/2) then carry the twiddles 1, w_2h^2j, w_2h^j, w_2h^3j,
// three general multiplies where two radix-2 stages take four.  Same
// positions as the radix-2 form, so the same output order.  An odd number
// of stages ends with one radix-2 stage (no twiddles).
// A length with one factor 3 (L = 3 P, P a power of two: 12, 24, 48) takes
// one radix-3 decimation-in-frequency step first: for j < P, with
// w = e^{-2 pi i / 3}, y_r(j) = x_j + w^r x_{j+P} + w^2r x_{j+2P} times
// w_L^{j r}, and X[3 m + r] is the P-point FFT of y_r; so element r P + p
// holds frequency 3 bitrev_P(p) + r (freq_of).
template <int L>
RRC_HD void fft_dif(float2 (&a)[L]) {
    if constexpr (L % 3 == 0) {
        constexpr int P = L / 3;
        constexpr float h3 = 0.86602540378443864676f;   // sqrt(3) / 2
#pragma unroll
        for (int j = 0; j < P; ++j) {
            const float2 a0 = a[j], a1 = a[j + P], a2 = a[j + 2 * P];
            const float2 sm = cadd(a1, a2), df = csub(a1, a2);
            const float2 t = make_float2(fmaf(-0.5f, sm.x, a0.x), fmaf(-0.5f, sm.y, a0.y));
            const float2 e = make_float2(h3 * df.y, -h3 * df.x);        // -i (sqrt3/2)(x_{j+P} - x_{j+2P})
            a[j] = cadd(a0, sm);
            a[j + P] = twmul<L>(cadd(t, e), j);
            a[j + 2 * P] = twmul<L>(csub(t, e), 2 * j);
        }
#pragma unroll
        for (int r = 0; r < 3; ++r) fft_dif<P>(*reinterpret_cast<float2(*)[P]>(&a[r * P]));
        return;
    }
#pragma unroll
    for (int h = L / 2; h >= 2; h >>= 2) {
        const int q = h / 2;
        const int tw = L / (2 * h);              // w_2h^m = w_L^{m tw}
#pragma unroll
        for (int b = 0; b < L; b += 2 * h) {
#pragma unroll
            for (int j = 0; j < q; ++j) {
                const float2 a0 = a[b + j], a1 = a[b + j + q], a2 = a[b + j + h], a3 = a[b + j + h + q];
                const float2 s02 = cadd(a0, a2), d02 = csub(a0, a2);
                const float2 s13 = cadd(a1, a3), d13 = csub(a1, a3);
                const float2 md13 = make_float2(d13.y, -d13.x);      // -i (a1 - a3)
                a[b + j] = cadd(s02, s13);
                a[b + j + q] = twmul<L>(csub(s02, s13), 2 * j * tw);
                a[b + j + h] = twmul<L>(cadd(d02, md13), j * tw);
                a[b + j + h + q] = twmul<L>(csub(d02, md13), 3 * j * tw);
            }
        }
    }
    if constexpr ((__builtin_ctz(L) & 1) != 0) {
#pragma unroll
        for (int b = 0; b < L; b += 2) {
            const float2 u = a[b], v = a[b + 1];
            a[b] = cadd(u, v);
            a[b + 1] = csub(u, v);
        }
    }
}

template <int L>
constexpr int bitrev(int r) {
    int out = 0;
    for (int m = 1, k = L >> 1; m < L; m <<= 1, k >>= 1)
        if (r & m) out |= k;
    return out;
}

// Frequency held by element r of fft_dif<L>'s output, and the element that
// holds frequency f (bit reversal for a power of two; for L = 3 P, element
// r' P + p holds 3 bitrev_P(p) + r').
template <int L>
constexpr int freq_of(int r) {
    if constexpr (L % 3 == 0) return 3 * bitrev<L / 3>(r % (L / 3)) + r / (L / 3);
    else return bitrev<L>(r);
}
template <int L>
constexpr int index_of(int f) {
    if constexpr (L % 3 == 0) return (f % 3) * (L / 3) + bitrev<L / 3>(f / 3);
    else return bitrev<L>(f);
}

constexpr int ilog2(int v) { return v <= 1 ? 0 : 1 + ilog2(v >> 1); }

// -------------------------------------------------------- wave reductions
//
// Sum over the 64 lanes of a wavefront, returned to every lane, in a fixed
// order (deterministic).  On the GPU: two quad permutations and two row
// rotations by DPP give every lane its 16-lane row sum, then the four row
// sums are read from lanes 0, 16, 32, 48.  Every lane must be active.

#ifdef RRC_HOST_EMU
template <typename T>
inline T wave_allsum(T v) {
    for (int o = 1; o <= 32; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}
template <typename T>
inline T wave_sum_last(T v) { return wave_allsum(v); }
inline float fast_rcp(float x) { return 1.0f / x; }
template <typename T>
inline T quad_sum(T v) {
    for (int o = 1; o <= 2; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}
template <typename T>
inline T row_sum(T v) {
    for (int o = 1; o <= 8; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}
template <typename T>
inline T oct_sum(T v) {
    for (int o = 1; o <= 4; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}
#else
template <int CTRL>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(dpp_i<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
    const int lo = dpp_i<CTRL>(__double2loint(v));
    const int hi = dpp_i<CTRL>(__double2hiint(v));
    return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane_f(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane_d(double v, int l) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), l),
                            __builtin_amdgcn_readlane(__double2loint(v), l));
}
__device__ __forceinline__ float wave_allsum(float v) {
    v += dpp_f<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_f<0x4E>(v);    // quad_perm [2,3,0,1]
    v += dpp_f<0x124>(v);   // row_ror:4
    v += dpp_f<0x128>(v);   // row_ror:8
    return (lane_f(v, 0) + lane_f(v, 16)) + (lane_f(v, 32) + lane_f(v, 48));
}
__device__ __forceinline__ double wave_allsum(double v) {
    v += dpp_d<0xB1>(v);
    v += dpp_d<0x4E>(v);
    v += dpp_d<0x124>(v);
    v += dpp_d<0x128>(v);
    return (lane_d(v, 0) + lane_d(v, 16)) + (lane_d(v, 32) + lane_d(v, 48));
}

// Reciprocal by the hardware approximation (v_rcp_f32, about 1 ulp).
__device__ __forceinline__ float fast_rcp(float x) { return __builtin_amdgcn_rcpf(x); }

// Sum over each quad of lanes / each row of 16 lanes, returned to every
// lane of the quad / row.
__device__ __forceinline__ float quad_sum(float v) {
    v += dpp_f<0xB1>(v);    // quad_perm [1,0,3,2]
    v += dpp_f<0x4E>(v);    // quad_perm [2,3,0,1]
    return v;
}
__device__ __forceinline__ float row_sum(float v) {
    v += dpp_f<0xB1>(v);
    v += dpp_f<0x4E>(v);
    v += dpp_f<0x124>(v);   // row_ror:4
    v += dpp_f<0x128>(v);   // row_ror:8
    return v;
}
__device__ __forceinline__ double quad_sum(double v) {
    v += dpp_d<0xB1>(v);
    v += dpp_d<0x4E>(v);
    return v;
}
__device__ __forceinline__ double row_sum(double v) {
    v += dpp_d<0xB1>(v);
    v += dpp_d<0x4E>(v);
    v += dpp_d<0x124>(v);
    v += dpp_d<0x128>(v);
    return v;
}
// Sum over each group of 8 lanes: the quad sums, then row_half_mirror
// (lane i of the group reads lane 7 - i, which lies in the other quad).
__device__ __forceinline__ float oct_sum(float v) {
    v += dpp_f<0xB1>(v);
    v += dpp_f<0x4E>(v);
    v += dpp_f<0x141>(v);   // row_half_mirror
    return v;
}
__device__ __forceinline__ double oct_sum(double v) {
    v += dpp_d<0xB1>(v);
    v += dpp_d<0x4E>(v);
    v += dpp_d<0x141>(v);
    return v;
}

// Sum over the 64 lanes, complete in lane 63 only (other lanes hold
// partial sums), kept in vector registers.  After the row sums, the
// row_bcast:15 step adds row 0 into row 1 and row 2 into row 3 (the other
// rows add zero), and row_bcast:31 adds rows 0+1 into rows 2 and 3.
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_rows_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xF, false);
}
__device__ __forceinline__ float wave_sum_last(float v) {
    v += dpp_f<0xB1>(v);
    v += dpp_f<0x4E>(v);
    v += dpp_f<0x124>(v);
    v += dpp_f<0x128>(v);
    v += __int_as_float(dpp_rows_i<0x142, 0xA>(__float_as_int(v)));   // row_bcast:15
    v += __int_as_float(dpp_rows_i<0x143, 0xC>(__float_as_int(v)));   // row_bcast:31
    return v;
}
__device__ __forceinline__ double wave_sum_last(double v) {
    v += dpp_d<0xB1>(v);
    v += dpp_d<0x4E>(v);
    v += dpp_d<0x124>(v);
    v += dpp_d<0x128>(v);
    v += __hiloint2double(dpp_rows_i<0x142, 0xA>(__double2hiint(v)), dpp_rows_i<0x142, 0xA>(__double2loint(v)));
    v += __hiloint2double(dpp_rows_i<0x143, 0xC>(__double2hiint(v)), dpp_rows_i<0x143, 0xC>(__double2loint(v)));
    return v;
}
#endif

// ------------------------------------------------------------- geometry

// The selected baseline-types of a plan, passed to kernels by value.
#ifndef RRC_HOST_EMU
// Per-unit completion stamps of a run: stamps[0] is the run's start and
// stamps[1 + u] the latest completion time of unit u's outputs, in ticks of
// the device's constant-rate wall clock.  Each stage that finishes a unit's
// outputs raises its entry (an atomic max on a vector memory path).
__device__ __forceinline__ void unit_done_stamp(unsigned long long* stamps, int unit) {
    atomicMax(stamps + 1 + unit, (unsigned long long)wall_clock64());
}
#endif

struct Sel {
    int n;                  // grid side
    int N;                  // n*n
    int K;                  // selected types
    int P;                  // pairs
    int dx[kMaxTypes];
    int dy[kMaxTypes];
    int off[kMaxTypes + 1]; // pair offset of each type, off[K] = P
};

// pair b of type t -> (i, j) with r_i - r_j = d_t
RRC_HD void pair_ij(const Sel& s, int t, int b_local, int& i, int& j) {
    const int dx = s.dx[t], dy = s.dy[t];
    const int w = s.n - (dx < 0 ? -dx : dx);
    const int yi = b_local / w + dy;
    const int xi = b_local % w + (dx > 0 ? dx : 0);
    i = yi * s.n + xi;
    j = i - (dy * s.n + dx);
}

// Global pair index of the pair (a, a - d_t) with antenna a = (ax, ay)
// first, or -1 if either antenna lies outside the grid.
RRC_HD int pair_as_first(const Sel& s, int t, int ax, int ay) {
    const int dx = s.dx[t], dy = s.dy[t];
    const int jx = ax - dx, jy = ay - dy;
    if (ax < 0 || ax >= s.n || ay < 0 || ay >= s.n) return -1;
    if (jx < 0 || jx >= s.n || jy < 0 || jy >= s.n) return -1;
    const int w = s.n - (dx < 0 ? -dx : dx);
    return s.off[t] + (ay - dy) * w + (ax - (dx > 0 ? dx : 0));
}

// Global pair index of the pair (a + d_t, a) with antenna a second, or -1.
RRC_HD int pair_as_second(const Sel& s, int t, int ax, int ay) {
    return pair_as_first(s, t, ax + s.dx[t], ay + s.dy[t]);
}

// type of global pair b (linear scan; K is small)
RRC_HD int type_of(const Sel& s, int b) {
    int t = 0;
    while (t + 1 < s.K && b >= s.off[t + 1]) ++t;
    return t;
}

}  // namespace rrc
