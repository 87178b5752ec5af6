// (a5) Reduced redundant-baseline calibration and (a6) the chi^2 adjoint.
//
// Model and objective: V_b = g_i conj(g_j) V_alpha for every selected pair
// (eq. redcal), chi^2 = sum_b |V_b - g_i conj(g_j) V_alpha|^2 (eq. redchi,
// uniform noise as in eq. noisecov), DoF = P - N - K + 2 (eq. dof).
//
// Solver (one workgroup per unit).  Gauss-Newton on the Taylor-expanded
// model (the paper's "Taylor expansion" linearisation, Sec. 2) written in
// multiplicative form: perturbing g_i -> g_i e^{eta_i} and
// V_alpha -> V_alpha e^{zeta_alpha} linearises the relative residual as
//     r_b / m_b  ~  eta_i + conj(eta_j) + zeta_alpha,   m_b = g_i conj(g_j) V_alpha,
// with weight |m_b|^2.  Its real part involves only log-amplitudes
// (a_i + a_j + c_alpha) and its imaginary part only phases
// (phi_i - phi_j + psi_alpha) -- the two real systems of eq. logcal, here
// with the current weights -- so each step solves two decoupled, sparse,
// positive semi-definite normal equations.  Their right-hand sides are the
// adjoint J^H r (the same sums as the chi^2 gradient of rrc_chisq_adj) and
// their diagonal is diag(J^H J); they are solved together by
// Jacobi-preconditioned conjugate gradients, matrix-free over the pairs.
//
// Precision: the first steps take the residual in FP32 from FP32
// parameters; once the rms log-step is below tol32 the parameters are
// promoted to FP64 and `fp64_steps` more steps take the residual in FP64
// (the normal equations stay FP32: iterative refinement).  The four
// degeneracies (Sec. 5.2) are fixed in FP64 and chi^2 is summed in FP64.
//
// Start (the paper does not say how its solver was started): either the
// caller's gains, or logcal amplitudes (real part of eq. logcal) with
// phases chained along the (1,0) and (0,1) groups.  V_alpha then starts at
// the group mean of V_b / (g_i conj(g_j)).
#include "rrc_device.h"
#include "rrc_launch.h"

#include <math.h>

namespace rrc {

constexpr int kSThreads = 256;
constexpr int kSWaves = kSThreads / 64;

__host__ __device__ inline size_t align16(size_t v) { return (v + 15) & ~(size_t)15; }

// Per-unit arrays.  "Hot" arrays are touched every CG iteration; they live
// in LDS when they fit, otherwise in the global slab.  "Cold" arrays are
// touched once per Gauss-Newton step and always live in the global slab.
struct HotLayout {
    size_t w, sa, sp, d, xa, ra, za, pa, qa, xp, rp, zp, pp, qp, bytes;
};
struct ColdLayout {
    size_t g, vm, gd, vmd, bytes;
};

__host__ __device__ inline HotLayout hot_layout(const Sel& s) {
    HotLayout L{};
    const size_t P = s.P, V = (size_t)s.N + s.K;
    size_t o = 0;
    L.w = o;  o = align16(o + 4 * P);
    L.sa = o; o = align16(o + 4 * P);
    L.sp = o; o = align16(o + 4 * P);
    size_t* vecs[] = {&L.d, &L.xa, &L.ra, &L.za, &L.pa, &L.qa, &L.xp, &L.rp, &L.zp, &L.pp, &L.qp};
    for (size_t* v : vecs) { *v = o; o = align16(o + 4 * V); }
    L.bytes = o;
    return L;
}
__host__ __device__ inline ColdLayout cold_layout(const Sel& s, size_t base) {
    ColdLayout L{};
    size_t o = base;
    L.g = o;   o = align16(o + 8 * (size_t)s.N);
    L.vm = o;  o = align16(o + 8 * (size_t)s.K);
    L.gd = o;  o = align16(o + 16 * (size_t)s.N);
    L.vmd = o; o = align16(o + 16 * (size_t)s.K);
    L.bytes = o - base;
    return L;
}

size_t solve_hot_bytes(const Sel& s) { return hot_layout(s).bytes; }
size_t solve_slab_bytes(const Sel& s, bool lds) {
    const size_t hot = lds ? 0 : hot_layout(s).bytes;
    return align16(hot + cold_layout(s, hot).bytes);
}
size_t solve_lds_bytes(const Sel& s, bool lds) { return lds ? hot_layout(s).bytes : 0; }

struct Mem {
    const Sel* ls;          // the selection copied to LDS, for type-indexed lookups
    float *w, *sa, *sp, *d;
    float *xa, *ra, *za, *pa, *qa;
    float *xp, *rp, *zp, *pp, *qp;
    float2* g;
    float2* vm;
    double2* gd;
    double2* vmd;
};

// ------------------------------------------------------------ reductions

struct Shared {
    Sel sel;                                // copy of the selection (runtime type indices)
    float bf[2 * kSWaves * 4];              // block_sum slots (two phases)
    double bd[2 * kSWaves * 12];
    double bcast[8];
};

// Sums NV values over the workgroup; every thread gets the totals, in a
// fixed order (deterministic).  The slots alternate between two phases, so
// one barrier suffices: a slot is rewritten only two calls later, after a
// barrier every reader of the previous use has passed.
struct Reducer {
    Shared* sh;
    int pf = 0, pd = 0;
};

template <int NV>
__device__ __forceinline__ void block_sum(float (&v)[NV], Reducer& R) {
    static_assert(NV <= 4, "float slots");
    float* slot = R.sh->bf + R.pf * (kSWaves * 4);
    R.pf ^= 1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = wave_allsum(v[i]);
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) slot[wave * 4 + i] = v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        float s = 0.f;
        for (int w = 0; w < kSWaves; ++w) s += slot[w * 4 + i];
        v[i] = s;
    }
}

template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], Reducer& R) {
    static_assert(NV <= 12, "double slots");
    double* slot = R.sh->bd + R.pd * (kSWaves * 12);
    R.pd ^= 1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = wave_allsum(v[i]);
    if (lane == 0) {
#pragma unroll
        for (int i = 0; i < NV; ++i) slot[wave * 12 + i] = v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        double s = 0.0;
        for (int w = 0; w < kSWaves; ++w) s += slot[w * 12 + i];
        v[i] = s;
    }
}

// --------------------------------------------------------- pair visitors
//
// Work-item tid owns antennas a = tid + k*NT (k < APT) and, for the type
// unknowns, type row t = 4*lane + wave (lane = tid % 64, wave = tid / 64)
// when that is < K.  Every pair is visited once from its first antenna.
// The selection is read from its LDS copy.  Type rows are summed by waves over each type's
// contiguous pair range (wave w takes types w, w+4, ...), and the owner lane
// of a type row is in the wave that sums it.

template <int APT>
struct Own {
    int a[APT], x[APT], y[APT];
    int trow;   // owned type row, or -1
};

template <int APT>
__device__ __forceinline__ Own<APT> own_antennas(const Sel& s) {
    Own<APT> o;
#pragma unroll
    for (int k = 0; k < APT; ++k) {
        o.a[k] = threadIdx.x + k * kSThreads;
        o.x[k] = o.a[k] % s.n;
        o.y[k] = o.a[k] / s.n;
    }
    const int t = (threadIdx.x & 63) * kSWaves + (threadIdx.x >> 6);
    o.trow = t < s.K ? t : -1;
    return o;
}

__device__ __forceinline__ float2 load_vred(const void* v, bool ci4, size_t idx) {
    if (ci4) {
        const int2 q = reinterpret_cast<const int2*>(v)[idx];
        return make_float2((float)q.x, (float)q.y);
    }
    return reinterpret_cast<const float2*>(v)[idx];
}
__device__ __forceinline__ double2 load_vred_d(const void* v, bool ci4, size_t idx) {
    if (ci4) {
        const int2 q = reinterpret_cast<const int2*>(v)[idx];
        return make_double2((double)q.x, (double)q.y);
    }
    const float2 f = reinterpret_cast<const float2*>(v)[idx];
    return make_double2(f.x, f.y);
}

// Antenna rows: out_a = sum over the pairs touching a of A_b (both ends),
// B_b (first end) - B_b (second end), and C_b (both ends, if C).
template <int APT>
__device__ __forceinline__ void gather_rows(const Sel& s, const Own<APT>& o, const float* A,
                                            const float* B, const float* C, float* outA,
                                            float* outB, float* outC) {
#pragma unroll
    for (int k = 0; k < APT; ++k) {
        if (o.a[k] >= s.N) continue;
        float ya = 0.f, yb = 0.f, yc = 0.f;
        for (int t = 0; t < s.K; ++t) {
            const int b1 = pair_as_first(s, t, o.x[k], o.y[k]);
            const int b2 = pair_as_second(s, t, o.x[k], o.y[k]);
            if (b1 >= 0) {
                ya += A[b1];
                yb += B[b1];
                if (C) yc += C[b1];
            }
            if (b2 >= 0) {
                ya += A[b2];
                yb -= B[b2];
                if (C) yc += C[b2];
            }
        }
        outA[o.a[k]] = ya;
        outB[o.a[k]] = yb;
        if (outC) outC[o.a[k]] = yc;
    }
}

// Type rows: out[N + t] = sum over the pairs of type t of A_b (and B_b, C_b).
template <int APT>
__device__ __forceinline__ void type_rows(const Sel& s, const float* A, const float* B, const float* C,
                                          float* outA, float* outB, float* outC) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int t = wave; t < s.K; t += kSWaves) {
        float ya = 0.f, yb = 0.f, yc = 0.f;
        for (int b = s.off[t] + lane; b < s.off[t + 1]; b += 64) {
            ya += A[b];
            yb += B[b];
            if (C) yc += C[b];
        }
        ya = wave_allsum(ya);
        yb = wave_allsum(yb);
        if (C) yc = wave_allsum(yc);
        if (lane == t / kSWaves) {
            outA[s.N + t] = ya;
            outB[s.N + t] = yb;
            if (outC) outC[s.N + t] = yc;
        }
    }
}

// ------------------------------------------------- matrix-free operators
//
// Amplitude system: rows b: a_i + a_j + c_t, weight w_b.
// Phase system:     rows b: p_i - p_j + c_t, weight w_b.
// H x = sum_b w_b row_b (row_b . x).  Computes qa = Ha pa, qp = Hp pp;
// each result element is written by its owner.
template <int APT>
__device__ __forceinline__ void apply_H(const Sel& s, const Own<APT>& o, const Mem& m) {
    const int N = s.N;
    for (int t = 0; t < s.K; ++t) {
        const int dxy = s.dy[t] * s.n + s.dx[t];
        const float cta = m.pa[N + t], ctp = m.pp[N + t];
#pragma unroll
        for (int k = 0; k < APT; ++k) {
            if (o.a[k] >= N) continue;
            const int b = pair_as_first(s, t, o.x[k], o.y[k]);
            if (b < 0) continue;
            const int i = o.a[k], j = i - dxy;
            const float wb = m.w[b];
            m.sa[b] = wb * (m.pa[i] + m.pa[j] + cta);
            m.sp[b] = wb * (m.pp[i] - m.pp[j] + ctp);
        }
    }
    __syncthreads();
    gather_rows<APT>(s, o, m.sa, m.sp, nullptr, m.qa, m.qp, nullptr);
    type_rows<APT>(*m.ls, m.sa, m.sp, nullptr, m.qa, m.qp, nullptr);
}

// Jacobi-preconditioned CG on both systems at once, from x = 0 with the
// right-hand sides already in ra / rp and the diagonal in d (inverted in
// place).  Returns the number of iterations, or -1 if a right-hand side is
// not finite.
template <int APT>
__device__ int pcg2(const Sel& s, const Own<APT>& o, const Mem& m, Reducer& R, int max_cg, float tol) {
    const int N = s.N;
    auto each = [&](auto&& f) {
#pragma unroll
        for (int k = 0; k < APT; ++k)
            if (o.a[k] < N) f(o.a[k]);
        if (o.trow >= 0) f(N + o.trow);
    };
    float v4[4] = {0.f, 0.f, 0.f, 0.f};
    each([&](int e) {
        const float di = m.d[e] > 0.f ? 1.0f / m.d[e] : 0.f;
        m.d[e] = di;                      // the diagonal is kept inverted from here on
        m.xa[e] = 0.f;
        m.xp[e] = 0.f;
        const float za = m.ra[e] * di, zp = m.rp[e] * di;
        m.pa[e] = za;
        m.pp[e] = zp;
        v4[0] += m.ra[e] * za;
        v4[1] += m.rp[e] * zp;
        v4[2] += m.ra[e] * m.ra[e];
        v4[3] += m.rp[e] * m.rp[e];
    });
    block_sum<4>(v4, R);
    if (!(v4[2] == v4[2]) || !(v4[3] == v4[3]) || isinf(v4[2]) || isinf(v4[3])) return -1;
    float rza = v4[0], rzp = v4[1];
    const float stopa = tol * tol * v4[2], stopp = tol * tol * v4[3];
    bool done_a = !(v4[2] > 0.f), done_p = !(v4[3] > 0.f);
    int it = 0;
    for (; it < max_cg && !(done_a && done_p); ++it) {
        apply_H<APT>(s, o, m);
        float v2[2] = {0.f, 0.f};
        each([&](int e) {
            v2[0] += m.pa[e] * m.qa[e];
            v2[1] += m.pp[e] * m.qp[e];
        });
        block_sum<2>(v2, R);
        const float ala = (!done_a && v2[0] > 0.f) ? rza / v2[0] : 0.f;
        const float alp = (!done_p && v2[1] > 0.f) ? rzp / v2[1] : 0.f;
        float w4[4] = {0.f, 0.f, 0.f, 0.f};
        float za_own[APT + 1], zp_own[APT + 1];
#pragma unroll
        for (int k = 0; k <= APT; ++k) {
            za_own[k] = zp_own[k] = 0.f;
            int e;
            if (k < APT) {
                e = o.a[k];
                if (e >= N) continue;
            } else {
                if (o.trow < 0) continue;
                e = N + o.trow;
            }
            const float di = m.d[e];
            m.xa[e] += ala * m.pa[e];
            m.xp[e] += alp * m.pp[e];
            const float ra = m.ra[e] - ala * m.qa[e];
            const float rp = m.rp[e] - alp * m.qp[e];
            m.ra[e] = ra;
            m.rp[e] = rp;
            const float za = ra * di, zp = rp * di;
            za_own[k] = za;
            zp_own[k] = zp;
            w4[0] += ra * za;
            w4[1] += rp * zp;
            w4[2] += ra * ra;
            w4[3] += rp * rp;
        }
        block_sum<4>(w4, R);
        const float ba = (rza > 0.f) ? w4[0] / rza : 0.f;
        const float bp = (rzp > 0.f) ? w4[1] / rzp : 0.f;
        if (!done_a) rza = w4[0];
        if (!done_p) rzp = w4[1];
#pragma unroll
        for (int k = 0; k <= APT; ++k) {
            int e;
            if (k < APT) {
                e = o.a[k];
                if (e >= N) continue;
            } else {
                if (o.trow < 0) continue;
                e = N + o.trow;
            }
            if (!done_a) m.pa[e] = za_own[k] + ba * m.pa[e];
            if (!done_p) m.pp[e] = zp_own[k] + bp * m.pp[e];
        }
        done_a = done_a || !(w4[2] > stopa);
        done_p = done_p || !(w4[3] > stopp);
        __syncthreads();
    }
    return it;
}

// ------------------------------------------------------------ GN pieces

// Residual pass, FP32: for every pair m_b, w_b = |m_b|^2 and
// q_b = r_b conj(m_b); then the right-hand sides (ra, rp = J^H r split into
// real and imaginary parts) and the diagonal d.
template <int APT>
__device__ void residual_pass32(const Sel& s, const Own<APT>& o, const Mem& m, const void* vred,
                                bool ci4, size_t vbase) {
    const int N = s.N;
    for (int t = 0; t < s.K; ++t) {
        const int dxy = s.dy[t] * s.n + s.dx[t];
        const float2 vt = m.vm[t];
#pragma unroll
        for (int k = 0; k < APT; ++k) {
            if (o.a[k] >= N) continue;
            const int b = pair_as_first(s, t, o.x[k], o.y[k]);
            if (b < 0) continue;
            const int i = o.a[k], j = i - dxy;
            const float2 mm = cmul(cmulc(m.g[i], m.g[j]), vt);
            const float2 q = cmulc(csub(load_vred(vred, ci4, vbase + b), mm), mm);
            m.sa[b] = q.x;
            m.sp[b] = q.y;
            m.w[b] = cabs2(mm);
        }
    }
    __syncthreads();
    gather_rows<APT>(s, o, m.sa, m.sp, m.w, m.ra, m.rp, m.d);
    type_rows<APT>(*m.ls, m.sa, m.sp, m.w, m.ra, m.rp, m.d);
}

// q_b = r_b conj(m_b) in FP64 for the pair (i, j) of type t.
__device__ __forceinline__ double2 q_hi(const Mem& m, const void* vred, bool ci4, size_t vb, int b,
                                        int i, int j, int t, double& wb) {
    const double2 mm = dmul(dmulc(m.gd[i], m.gd[j]), m.vmd[t]);
    wb = dabs2(mm);
    return dmulc(dsub(load_vred_d(vred, ci4, vb + b), mm), mm);
}

// Residual pass, FP64: near the optimum J^H r is a sum of per-pair terms
// of the size of the noise that cancel to a tiny total, so it is summed in
// FP64: per antenna over its pairs, and per type by the summing wave, each
// pair's residual recomputed where it is needed.  The FP32 normal
// equations then get the right-hand side scaled to unit norm; the scale is
// returned (multiply the solution by it).
template <int APT>
__device__ double residual_pass64(const Sel& s, const Own<APT>& o, const Mem& m, Reducer& R,
                                  const void* vred, bool ci4, size_t vbase) {
    const int N = s.N;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int t = 0; t < s.K; ++t) {
        const int dxy = s.dy[t] * s.n + s.dx[t];
#pragma unroll
        for (int k = 0; k < APT; ++k) {
            if (o.a[k] >= N) continue;
            const int b = pair_as_first(s, t, o.x[k], o.y[k]);
            if (b < 0) continue;
            const int i = o.a[k];
            const double2 mm = dmul(dmulc(m.gd[i], m.gd[i - dxy]), m.vmd[t]);
            m.w[b] = (float)dabs2(mm);
        }
    }
    __syncthreads();
    double ra_loc[APT + 1], rp_loc[APT + 1];
    double nrm[1] = {0.0};
#pragma unroll
    for (int k = 0; k < APT; ++k) {
        ra_loc[k] = rp_loc[k] = 0.0;
        if (o.a[k] >= N) continue;
        const int a = o.a[k];
        double ya = 0.0, yp = 0.0;
        float dd = 0.f;
        for (int t = 0; t < s.K; ++t) {
            const int dxy = s.dy[t] * s.n + s.dx[t];
            const int b1 = pair_as_first(s, t, o.x[k], o.y[k]);
            const int b2 = pair_as_second(s, t, o.x[k], o.y[k]);
            double wb;
            if (b1 >= 0) {
                const double2 q = q_hi(m, vred, ci4, vbase, b1, a, a - dxy, t, wb);
                ya += q.x;
                yp += q.y;
                dd += m.w[b1];
            }
            if (b2 >= 0) {
                const double2 q = q_hi(m, vred, ci4, vbase, b2, a + dxy, a, t, wb);
                ya += q.x;
                yp -= q.y;
                dd += m.w[b2];
            }
        }
        ra_loc[k] = ya;
        rp_loc[k] = yp;
        m.d[a] = dd;
        nrm[0] += ya * ya + yp * yp;
    }
    ra_loc[APT] = rp_loc[APT] = 0.0;
    const Sel& ls = *m.ls;
    for (int t = wave; t < ls.K; t += kSWaves) {
        double ya = 0.0, yp = 0.0;
        float dd = 0.f;
        for (int b = ls.off[t] + lane; b < ls.off[t + 1]; b += 64) {
            int i, j;
            pair_ij(ls, t, b - ls.off[t], i, j);
            double wb;
            const double2 q = q_hi(m, vred, ci4, vbase, b, i, j, t, wb);
            ya += q.x;
            yp += q.y;
            dd += m.w[b];
        }
        ya = wave_allsum(ya);
        yp = wave_allsum(yp);
        dd = wave_allsum(dd);
        if (lane == t / kSWaves) {
            ra_loc[APT] = ya;
            rp_loc[APT] = yp;
            m.d[N + t] = dd;
            nrm[0] += ya * ya + yp * yp;
        }
    }
    block_sum<1>(nrm, R);
    const double scale = nrm[0] > 0.0 ? sqrt(nrm[0]) : 1.0;
    const double inv = 1.0 / scale;
#pragma unroll
    for (int k = 0; k < APT; ++k) {
        if (o.a[k] >= N) continue;
        m.ra[o.a[k]] = (float)(ra_loc[k] * inv);
        m.rp[o.a[k]] = (float)(rp_loc[k] * inv);
    }
    if (o.trow >= 0) {
        m.ra[N + o.trow] = (float)(ra_loc[APT] * inv);
        m.rp[N + o.trow] = (float)(rp_loc[APT] * inv);
    }
    return scale;
}

// V_t = mean over the group of V_b / (g_i conj(g_j)) (FP32 parameters),
// summed by the waves; visible to all after the closing barrier.
template <int APT>
__device__ void group_mean(const Mem& m, const void* vred, bool ci4, size_t vbase) {
    const Sel& s = *m.ls;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int t = wave; t < s.K; t += kSWaves) {
        float sr = 0.f, si = 0.f;
        for (int b = s.off[t] + lane; b < s.off[t + 1]; b += 64) {
            int i, j;
            pair_ij(s, t, b - s.off[t], i, j);
            const float2 gg = cmulc(m.g[i], m.g[j]);
            const float2 q = cmulc(load_vred(vred, ci4, vbase + b), gg);
            const float inv = 1.0f / cabs2(gg);
            sr += q.x * inv;
            si += q.y * inv;
        }
        sr = wave_allsum(sr);
        si = wave_allsum(si);
        if (lane == 0) {
            const float cnt = (float)(s.off[t + 1] - s.off[t]);
            m.vm[t] = make_float2(sr / cnt, si / cnt);
        }
    }
    __syncthreads();
}

// Logcal amplitudes and chained phases (see the file comment).
template <int APT>
__device__ void firstcal(const Sel& s, const Own<APT>& o, const Mem& m, Reducer& R, const void* vred,
                         bool ci4, size_t vbase, int t10, int t01, int max_cg) {
    const int N = s.N, n = s.n;
    // amplitude: unweighted least squares on ln|V_b|
    for (int t = 0; t < s.K; ++t) {
#pragma unroll
        for (int k = 0; k < APT; ++k) {
            if (o.a[k] >= N) continue;
            const int b = pair_as_first(s, t, o.x[k], o.y[k]);
            if (b < 0) continue;
            m.sa[b] = 0.5f * logf(fmaxf(cabs2(load_vred(vred, ci4, vbase + b)), 1e-30f));
            m.sp[b] = 0.f;
            m.w[b] = 1.0f;
        }
    }
    __syncthreads();
    gather_rows<APT>(s, o, m.sa, m.sp, m.w, m.ra, m.rp, m.d);
    type_rows<APT>(*m.ls, m.sa, m.sp, m.w, m.ra, m.rp, m.d);
    pcg2<APT>(s, o, m, R, max_cg, 1e-3f);
    // phase increments along the chains, in qp[] (scratch)
    const int off10 = m.ls->off[t10], off01 = m.ls->off[t01];
    const float2 v10 = load_vred(vred, ci4, vbase + off10);
    const float2 v01 = load_vred(vred, ci4, vbase + off01);
    const float psi10 = atan2f(v10.y, v10.x), psi01 = atan2f(v01.y, v01.x);
    const float2 r10 = make_float2(cosf(psi10), -sinf(psi10));
    const float2 r01 = make_float2(cosf(psi01), -sinf(psi01));
#pragma unroll
    for (int k = 0; k < APT; ++k) {
        if (o.a[k] >= N) continue;
        const int x = o.x[k], y = o.y[k];
        float inc = 0.f;
        if (y == 0 && x >= 1) {
            const float2 v = cmul(load_vred(vred, ci4, vbase + off10 + (x - 1)), r10);
            inc = atan2f(v.y, v.x);
        } else if (y >= 1) {
            const float2 v = cmul(load_vred(vred, ci4, vbase + off01 + (y - 1) * n + x), r01);
            inc = atan2f(v.y, v.x);
        }
        m.qp[o.a[k]] = inc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        m.qp[0] = 0.f;
        for (int x = 1; x < n; ++x) m.qp[x] += m.qp[x - 1];
    }
    __syncthreads();
    if ((int)threadIdx.x < n) {
        const int x = threadIdx.x;
        for (int y = 1; y < n; ++y) m.qp[y * n + x] += m.qp[(y - 1) * n + x];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < APT; ++k) {
        if (o.a[k] >= N) continue;
        const float amp = expf(m.xa[o.a[k]]);
        float sn, cs;
        sincosf(m.qp[o.a[k]], &sn, &cs);
        m.g[o.a[k]] = make_float2(amp * cs, amp * sn);
    }
    __syncthreads();
}

// ------------------------------------------------------------- the kernel

// The whole solve of one unit by one workgroup.
template <int APT, bool LDS>
__device__ void solve_unit(const SolveLaunch& L, Shared& sh, unsigned char* ssm, int unit) {
    // The selection is read from an LDS copy: indexing the by-value kernel
    // argument with a type index would make the compiler copy the argument
    // to private memory.
    if (threadIdx.x == 0) {
        const int* src = reinterpret_cast<const int*>(&L.sel);
        int* dst = reinterpret_cast<int*>(&sh.sel);
#pragma unroll
        for (int i = 0; i < (int)(sizeof(Sel) / sizeof(int)); ++i) dst[i] = src[i];
    }
    __syncthreads();
    const Sel& ls = sh.sel;
    const Sel& s = ls;
    Reducer R{&sh};
    const int N = s.N, K = s.K;
    const size_t vbase = (size_t)unit * s.P;
    char* slab = L.slab + (size_t)unit * L.slab_bytes;
    char* hot = LDS ? reinterpret_cast<char*>(ssm) : slab;
    const HotLayout H = hot_layout(s);
    const ColdLayout C = cold_layout(s, LDS ? 0 : H.bytes);
    Mem m;
    m.ls = &ls;
    m.w = reinterpret_cast<float*>(hot + H.w);
    m.sa = reinterpret_cast<float*>(hot + H.sa);
    m.sp = reinterpret_cast<float*>(hot + H.sp);
    m.d = reinterpret_cast<float*>(hot + H.d);
    m.xa = reinterpret_cast<float*>(hot + H.xa);
    m.ra = reinterpret_cast<float*>(hot + H.ra);
    m.za = reinterpret_cast<float*>(hot + H.za);
    m.pa = reinterpret_cast<float*>(hot + H.pa);
    m.qa = reinterpret_cast<float*>(hot + H.qa);
    m.xp = reinterpret_cast<float*>(hot + H.xp);
    m.rp = reinterpret_cast<float*>(hot + H.rp);
    m.zp = reinterpret_cast<float*>(hot + H.zp);
    m.pp = reinterpret_cast<float*>(hot + H.pp);
    m.qp = reinterpret_cast<float*>(hot + H.qp);
    m.g = reinterpret_cast<float2*>(slab + C.g);
    m.vm = reinterpret_cast<float2*>(slab + C.vm);
    m.gd = reinterpret_cast<double2*>(slab + C.gd);
    m.vmd = reinterpret_cast<double2*>(slab + C.vmd);

    const Own<APT> o = own_antennas<APT>(s);
    const SolveOpts& op = L.o;

    // ---- start
    if (op.init_mode == 1 && L.gains_in) {
#pragma unroll
        for (int k = 0; k < APT; ++k)
            if (o.a[k] < N) m.g[o.a[k]] = L.gains_in[(size_t)unit * N + o.a[k]];
        __syncthreads();
    } else {
        int t10 = -1, t01 = -1;
        for (int t = 0; t < K; ++t) {
            if (ls.dx[t] == 1 && ls.dy[t] == 0) t10 = t;
            if (ls.dx[t] == 0 && ls.dy[t] == 1) t01 = t;
        }
        firstcal<APT>(s, o, m, R, L.vred, L.ci4, vbase, t10, t01, op.max_cg);
    }
    group_mean<APT>(m, L.vred, L.ci4, vbase);

    // ---- Gauss-Newton
    int status = 0;
    int steps = 0;
    bool hi = false;
    int hi_left = op.fp64_steps;
    int n32 = 0;
    while (true) {
        double xscale = 1.0;
        if (hi) {
            if (hi_left <= 0) break;
            xscale = residual_pass64<APT>(s, o, m, R, L.vred, L.ci4, vbase);
        } else {
            residual_pass32<APT>(s, o, m, L.vred, L.ci4, vbase);
        }
        if (pcg2<APT>(s, o, m, R, op.max_cg, op.cg_tol) < 0) {   // non-finite data
            status = 2;
            break;
        }
        // update g <- g e^{eta}, V <- V e^{zeta}
        float e2[1] = {0.f};
#pragma unroll
        for (int k = 0; k <= APT; ++k) {
            int e;
            if (k < APT) {
                e = o.a[k];
                if (e >= N) continue;
            } else {
                if (o.trow < 0) continue;
                e = N + o.trow;
            }
            const float xa = m.xa[e], xp = m.xp[e];
            if (hi) {
                const double xad = xa * xscale, xpd = xp * xscale;
                e2[0] += (float)(xad * xad + xpd * xpd);
                double sn, cs;
                sincos(xpd, &sn, &cs);
                const double amp = exp(xad);
                const double2 f = make_double2(amp * cs, amp * sn);
                if (e < N) {
                    m.gd[e] = dmul(m.gd[e], f);
                    m.g[e] = to_f(m.gd[e]);
                } else {
                    m.vmd[e - N] = dmul(m.vmd[e - N], f);
                    m.vm[e - N] = to_f(m.vmd[e - N]);
                }
            } else {
                e2[0] += xa * xa + xp * xp;
                float sn, cs;
                sincosf(xp, &sn, &cs);
                const float amp = expf(xa);
                const float2 f = make_float2(amp * cs, amp * sn);
                if (e < N) m.g[e] = cmul(m.g[e], f);
                else m.vm[e - N] = cmul(m.vm[e - N], f);
            }
        }
        block_sum<1>(e2, R);
        ++steps;
        const float rms = sqrtf(e2[0] / (float)(N + K));
        if (!(rms == rms) || isinf(rms)) {
            status = 2;
            break;
        }
        if (hi) {
            --hi_left;
        } else {
            ++n32;
            if (rms < op.tol32 || n32 >= op.max_gn) {
                if (!(rms < op.tol32)) status = 1;
                hi = true;
#pragma unroll
                for (int k = 0; k < APT; ++k)
                    if (o.a[k] < N) m.gd[o.a[k]] = to_d(m.g[o.a[k]]);
                if ((int)threadIdx.x < K) m.vmd[threadIdx.x] = to_d(m.vm[threadIdx.x]);
                __syncthreads();
            }
        }
    }
    if (!hi) {
#pragma unroll
        for (int k = 0; k < APT; ++k)
            if (o.a[k] < N) m.gd[o.a[k]] = to_d(m.g[o.a[k]]);
        if ((int)threadIdx.x < K) m.vmd[threadIdx.x] = to_d(m.vm[threadIdx.x]);
        __syncthreads();
    }

    // ---- degeneracies (FP64)
    if (op.degen_mode == 1 && L.gains_ref) {
        double v9[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int k = 0; k < APT; ++k) {
            if (o.a[k] >= N) continue;
            const double2 g = m.gd[o.a[k]];
            const double2 gr = to_d(L.gains_ref[(size_t)unit * N + o.a[k]]);
            const double2 q = dmulc(g, gr);
            const double ph = atan2(q.y, q.x);
            const double x = o.x[k], y = o.y[k];
            v9[0] += 0.5 * log(dabs2(g)) - 0.5 * log(dabs2(gr));
            v9[1] += ph;
            v9[2] += ph * x;
            v9[3] += ph * y;
            v9[4] += x;
            v9[5] += y;
            v9[6] += x * x;
            v9[7] += x * y;
            v9[8] += y * y;
        }
        block_sum<9>(v9, R);
        if (threadIdx.x == 0) {
            // [N  Sx  Sy ; Sx Sxx Sxy ; Sy Sxy Syy] c = [S, Sx, Sy] by Cramer's rule
            const double a00 = N, a01 = v9[4], a02 = v9[5], a11 = v9[6], a12 = v9[7], a22 = v9[8];
            const double det = a00 * (a11 * a22 - a12 * a12) - a01 * (a01 * a22 - a12 * a02) +
                               a02 * (a01 * a12 - a11 * a02);
            const double b0 = v9[1], b1 = v9[2], b2 = v9[3];
            const double c0 = (b0 * (a11 * a22 - a12 * a12) - a01 * (b1 * a22 - a12 * b2) +
                               a02 * (b1 * a12 - a11 * b2)) / det;
            const double c1 = (a00 * (b1 * a22 - a12 * b2) - b0 * (a01 * a22 - a12 * a02) +
                               a02 * (a01 * b2 - b1 * a02)) / det;
            const double c2 = (a00 * (a11 * b2 - b1 * a12) - a01 * (a01 * b2 - b1 * a02) +
                               b0 * (a01 * a12 - a11 * a02)) / det;
            sh.bcast[0] = exp(v9[0] / N);
            sh.bcast[1] = c0;
            sh.bcast[2] = c1;
            sh.bcast[3] = c2;
        }
    } else {
        double v1[1] = {0.0};
#pragma unroll
        for (int k = 0; k < APT; ++k)
            if (o.a[k] < N) v1[0] += 0.5 * log(dabs2(m.gd[o.a[k]]));
        block_sum<1>(v1, R);
        if (threadIdx.x == 0) {
            const double2 g0 = m.gd[0], g1 = m.gd[1], gn = m.gd[s.n];
            const double2 qx = dmulc(g1, g0), qy = dmulc(gn, g0);
            sh.bcast[0] = exp(v1[0] / N);
            sh.bcast[1] = atan2(g0.y, g0.x);
            sh.bcast[2] = atan2(qx.y, qx.x);
            sh.bcast[3] = atan2(qy.y, qy.x);
        }
    }
    __syncthreads();
    {
        const double lam = sh.bcast[0], c0 = sh.bcast[1], kx = sh.bcast[2], ky = sh.bcast[3];
#pragma unroll
        for (int k = 0; k < APT; ++k) {
            if (o.a[k] >= N) continue;
            double sn, cs;
            sincos(-(c0 + kx * o.x[k] + ky * o.y[k]), &sn, &cs);
            const double2 g = m.gd[o.a[k]];
            m.gd[o.a[k]] = make_double2((g.x * cs - g.y * sn) / lam, (g.x * sn + g.y * cs) / lam);
        }
        if ((int)threadIdx.x < K) {
            const int t = threadIdx.x;
            double sn, cs;
            sincos(kx * ls.dx[t] + ky * ls.dy[t], &sn, &cs);
            const double2 v = m.vmd[t];
            const double l2 = lam * lam;
            m.vmd[t] = make_double2((v.x * cs - v.y * sn) * l2, (v.x * sn + v.y * cs) * l2);
        }
    }
    __syncthreads();

    // ---- chi^2 (FP64) and outputs
    double c1[1] = {0.0};
    for (int t = 0; t < K; ++t) {
        const int dxy = s.dy[t] * s.n + s.dx[t];
#pragma unroll
        for (int k = 0; k < APT; ++k) {
            if (o.a[k] >= N) continue;
            const int b = pair_as_first(s, t, o.x[k], o.y[k]);
            if (b < 0) continue;
            const int i = o.a[k], j = i - dxy;
            const double2 mm = dmul(dmulc(m.gd[i], m.gd[j]), m.vmd[t]);
            c1[0] += dabs2(dsub(load_vred_d(L.vred, L.ci4, vbase + b), mm));
        }
    }
    block_sum<1>(c1, R);
#pragma unroll
    for (int k = 0; k < APT; ++k)
        if (o.a[k] < N) L.gains_out[(size_t)unit * N + o.a[k]] = to_f(m.gd[o.a[k]]);
    if ((int)threadIdx.x < K) L.vmodel[(size_t)unit * K + threadIdx.x] = to_f(m.vmd[threadIdx.x]);
    if (threadIdx.x == 0) {
        const bool fin = c1[0] == c1[0] && !isinf(c1[0]);
        L.chisq[unit] = (float)c1[0];
        L.niter[unit] = steps;
        L.status[unit] = fin ? status : 2;
    }
}

#ifndef RRC_HOST_EMU
template <int APT, bool LDS>
__global__ __launch_bounds__(kSThreads) void k_solve(SolveLaunch L) {
    extern __shared__ __align__(16) unsigned char ssm[];
    __shared__ Shared sh;
    solve_unit<APT, LDS>(L, sh, ssm, blockIdx.x);
}

template <int APT, bool LDS_OK>
static hipError_t launch_solve_apt(const SolveLaunch& L, hipStream_t st) {
    if constexpr (LDS_OK) {
        if (L.lds) {
            auto kern = k_solve<APT, true>;
            (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.lds_bytes);
            hipLaunchKernelGGL(kern, dim3(L.n_units), dim3(kSThreads), L.lds_bytes, st, L);
            return hipGetLastError();
        }
    } else {
        if (L.lds) return hipErrorInvalidValue;
    }
    hipLaunchKernelGGL((k_solve<APT, false>), dim3(L.n_units), dim3(kSThreads), 0, st, L);
    return hipGetLastError();
}

hipError_t launch_solve(const SolveLaunch& L, hipStream_t st) {
    const int apt = (L.sel.N + kSThreads - 1) / kSThreads;
    if (apt <= 1) return launch_solve_apt<1, true>(L, st);
    if (apt <= 2) return launch_solve_apt<2, true>(L, st);
    if (apt <= 4) return launch_solve_apt<4, true>(L, st);
    if (apt <= 16) return launch_solve_apt<16, false>(L, st);
    return hipErrorInvalidValue;
}

// --------------------------------------------------- chi^2 and its adjoint
//
// One workgroup per unit.  Forward: sum_b |r_b|^2 in FP64 over FP32
// products.  Adjoint (a6): antenna-centric gathers over the 2K incident
// pairs, r_b recomputed on the fly; type sums by wave reductions.

template <int APT, bool ADJ>
__global__ __launch_bounds__(kSThreads) void k_chisq(ChisqLaunch L) {
    __shared__ Shared sh;
    if (threadIdx.x == 0) {
        const int* src = reinterpret_cast<const int*>(&L.sel);
        int* dst = reinterpret_cast<int*>(&sh.sel);
#pragma unroll
        for (int i = 0; i < (int)(sizeof(Sel) / sizeof(int)); ++i) dst[i] = src[i];
    }
    __syncthreads();
    const Sel& s = sh.sel;
    const int unit = blockIdx.x;
    const int N = s.N, K = s.K;
    const float2* g = L.g + (size_t)unit * N;
    const float2* vm = L.vm + (size_t)unit * K;
    const float2* vr = L.vred + (size_t)unit * s.P;
    const Own<APT> o = own_antennas<APT>(s);
    Reducer R{&sh};
    if constexpr (!ADJ) {
        double c1[1] = {0.0};
        for (int t = 0; t < K; ++t) {
            const int dxy = s.dy[t] * s.n + s.dx[t];
#pragma unroll
            for (int k = 0; k < APT; ++k) {
                if (o.a[k] >= N) continue;
                const int b = pair_as_first(s, t, o.x[k], o.y[k]);
                if (b < 0) continue;
                const int i = o.a[k], j = i - dxy;
                const float2 r = csub(vr[b], cmul(cmulc(g[i], g[j]), vm[t]));
                c1[0] += (double)cabs2(r);
            }
        }
        block_sum<1>(c1, R);
        if (threadIdx.x == 0) L.chisq[unit] = (float)c1[0];
    } else {
        // antenna rows
#pragma unroll
        for (int k = 0; k < APT; ++k) {
            if (o.a[k] >= N) continue;
            const int a = o.a[k];
            float2 gr = make_float2(0.f, 0.f);
            float dg = 0.f;
            for (int t = 0; t < K; ++t) {
                const int dxy = s.dy[t] * s.n + s.dx[t];
                const int b1 = pair_as_first(s, t, o.x[k], o.y[k]);
                if (b1 >= 0) {   // pair (a, j): - r_b g_j conj(V_t)
                    const int j = a - dxy;
                    const float2 c = cmulc(g[j], vm[t]);            // g_j conj(V_t)
                    const float2 r = csub(vr[b1], cmul(cmulc(g[a], g[j]), vm[t]));
                    gr = csub(gr, cmul(r, c));
                    dg += cabs2(c);
                }
                const int b2 = pair_as_second(s, t, o.x[k], o.y[k]);
                if (b2 >= 0) {   // pair (i, a): - conj(r_b) g_i V_t
                    const int i = a + dxy;
                    const float2 c = cmul(g[i], vm[t]);
                    const float2 r = csub(vr[b2], cmul(cmulc(g[i], g[a]), vm[t]));
                    gr = csub(gr, cmul(cconj(r), c));
                    dg += cabs2(c);
                }
            }
            if (L.grad_g) L.grad_g[(size_t)unit * N + a] = make_float2(2.f * gr.x, 2.f * gr.y);
            if (L.diag_g) L.diag_g[(size_t)unit * N + a] = dg;
        }
        // type rows, summed by the waves over each type's pairs
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        for (int t = wave; t < K; t += kSWaves) {
            float sr = 0.f, si = 0.f, sd = 0.f;
            for (int b = s.off[t] + lane; b < s.off[t + 1]; b += 64) {
                int i, j;
                pair_ij(s, t, b - s.off[t], i, j);
                const float2 gg = cmulc(g[j], g[i]);                // conj(g_i) g_j
                const float2 r = csub(vr[b], cmul(cmulc(g[i], g[j]), vm[t]));
                const float2 q = cmul(r, gg);
                sr -= q.x;
                si -= q.y;
                sd += cabs2(gg);
            }
            sr = wave_allsum(sr);
            si = wave_allsum(si);
            sd = wave_allsum(sd);
            if (lane == 0) {
                if (L.grad_v) L.grad_v[(size_t)unit * K + t] = make_float2(2.f * sr, 2.f * si);
                if (L.diag_v) L.diag_v[(size_t)unit * K + t] = sd;
            }
        }
    }
}

template <int APT>
static hipError_t launch_chisq_apt(const ChisqLaunch& L, hipStream_t st, bool adj) {
    if (adj) hipLaunchKernelGGL((k_chisq<APT, true>), dim3(L.n_units), dim3(kSThreads), 0, st, L);
    else hipLaunchKernelGGL((k_chisq<APT, false>), dim3(L.n_units), dim3(kSThreads), 0, st, L);
    return hipGetLastError();
}

hipError_t launch_chisq(const ChisqLaunch& L, hipStream_t st, bool adjoint) {
    const int apt = (L.sel.N + kSThreads - 1) / kSThreads;
    if (apt <= 1) return launch_chisq_apt<1>(L, st, adjoint);
    if (apt <= 2) return launch_chisq_apt<2>(L, st, adjoint);
    if (apt <= 4) return launch_chisq_apt<4>(L, st, adjoint);
    if (apt <= 8) return launch_chisq_apt<8>(L, st, adjoint);
    if (apt <= 16) return launch_chisq_apt<16>(L, st, adjoint);
    return hipErrorInvalidValue;
}

#endif  // RRC_HOST_EMU

}  // namespace rrc
