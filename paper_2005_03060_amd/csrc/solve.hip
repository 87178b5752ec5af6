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
// with weight w_b = |m_b|^2 = |g_i|^2 |g_j|^2 |V_alpha|^2.  Its real part
// involves only log-amplitudes (a_i + a_j + c_alpha) and its imaginary part
// only phases (phi_i - phi_j + psi_alpha) -- the two real systems of
// eq. logcal, here with the current weights -- so each step solves two
// decoupled, sparse, positive semi-definite normal equations.  Their
// right-hand sides are the adjoint J^H r (the sums of rrc_chisq_adj) and
// their diagonal is diag(J^H J); both are solved together by
// Jacobi-preconditioned conjugate gradients, matrix-free.
//
// Layout.  Work-item a owns antenna row a (and a + NT, ... when the grid
// has more antennas than the workgroup has work-items); work-item t < K
// also owns type row t.  A work-item keeps the CG state of its rows in
// registers.  The only vector other work-items read is the search
// direction, kept in LDS as one 16-byte record per row
// {p_amp, p_phase, |g|^2 (|V|^2 for a type row), -}: the matrix-vector
// product of an antenna row needs one LDS read per incident pair (at most
// 2K) and no per-pair storage, so the whole state of a unit (directions,
// gains and unique visibilities) fits in LDS for any grid up to 64 x 64.  Type-row
// sums (over a type's pairs) and CG's dot products are block reductions in
// a fixed order, so results are deterministic.
//
// Precision: parameters, residuals and the right-hand side are FP64; the
// right-hand side is handed to the FP32 normal equations scaled to unit
// norm, so each step is one step of iterative refinement (near the optimum
// J^H r is a sum of terms the size of the noise that cancel to a tiny
// total, which FP32 could not resolve).  Steps continue until the rms
// log-step is below tol32 (at most max_gn), then `fp64_steps` more.  The
// four degeneracies (Sec. 5.2) are fixed in FP64 and chi^2 is summed in
// FP64.
//
// Start (the paper does not say how its solver was started): either the
// caller's gains, or logcal amplitudes (real part of eq. logcal, unit
// weights) with phases chained along the (1,0) and (0,1) groups.  V_alpha
// then starts at the group mean of V_b / (g_i conj(g_j)).
#include "rrc_device.h"
#include "rrc_launch.h"

#include <math.h>

namespace rrc {

constexpr int kChunk = 8;                     // types per FP64 type-sum reduction
constexpr size_t kLdsPerCu = 160 * 1024;      // LDS of one gfx950 CU

__host__ __device__ inline size_t align16(size_t v) { return (v + 15) & ~(size_t)15; }

// Dynamic LDS of one unit's solve.
// Parameters are held in FP64 throughout; in the FP32 phase they carry
// FP32 values (exactly) and are read and updated in FP32.
// With vcache the unit's V^reduced (8 bytes per pair, as stored: complex64
// or the 4-bit path's int32 pairs) follows, read once from HBM instead of
// at every residual pass.
struct SolveLayout {
    size_t rec, gd, vmd, vr, bytes;
};
__host__ __device__ inline SolveLayout solve_layout(const Sel& s, bool vcache) {
    SolveLayout L{};
    size_t o = 0;
    L.rec = o; o = align16(o + 16 * ((size_t)s.N + s.K));
    L.gd = o;  o = align16(o + 16 * (size_t)s.N);
    L.vmd = o; o = align16(o + 16 * (size_t)s.K);
    L.vr = o;  if (vcache) o = align16(o + 8 * (size_t)s.P);
    L.bytes = o;
    return L;
}

size_t solve_lds_bytes(const Sel& s, bool vcache) { return solve_layout(s, vcache).bytes; }

// Workgroup shape: one antenna per work-item up to 512 antennas, then
// 512 work-items with 2, 4, 5 or 8 antennas each.
inline int solve_threads_for(int N) { return N <= 256 ? 256 : 512; }

// Per-type constants of the selection, in LDS: the raster offset d_t of
// the type and the pair indices as affine functions of an antenna's
// (x, y): pair (a, a - d_t) is c1 + y w + x, pair (a + d_t, a) is
// c2 + y w + x (a pair type's group is stored row-major over the rows of
// its first antenna, w = n - |dx| pairs per row).
struct TypeInfo {
    int dxy, w, c1, c2;
    int dx, dy, off, cnt;
};

// ------------------------------------------------------------ reductions
//
// block_sum adds NV values over the workgroup and returns the totals to
// every work-item, in a fixed order (deterministic), with few
// instructions per wave: DPP sums over Q lanes; the P = NT / Q partials of
// each value go to LDS laid out [value][partial]; per value, 16 (or 8)
// lanes add a share of them each and a DPP sum over those lanes; the
// totals go back through LDS.  Two
// barriers.  Consecutive calls may reuse the buffers: a work-item writes
// the next call's partials only after the previous call's second barrier,
// which every reader of its partials has passed, and writes totals only
// after the next call's first barrier, which every reader of the previous
// totals has passed.  Float and double reductions share the buffers.
template <int NT, typename T>
struct RedGeom {
    static constexpr int Q = sizeof(T) == 4 ? (NT <= 256 ? 1 : (NT <= 512 ? 4 : 16))
                                            : (NT <= 256 ? 4 : 64);
    static constexpr int P = NT / Q;
    // row stride of the partials in LDS: 64 bytes of padding, so that the
    // second stage's lane groups (32 consecutive words each) start 16 banks
    // apart and a wave's reads take the minimum number of passes
    static constexpr int PS = P + 64 / (int)sizeof(T);
};
constexpr int kRedNF = 2 * kMaxTypes + 6;     // floats per reduction (max)
constexpr int kRedND = 3 * kChunk + 1;        // doubles per reduction (max)

template <int NT>
constexpr int red_bytes() {
    constexpr int f = kRedNF * RedGeom<NT, float>::PS * 4 + kRedNF * 4;
    constexpr int d = kRedND * RedGeom<NT, double>::PS * 8 + kRedND * 8;
    return f > d ? f : d;
}

template <int NW>
struct Shared {
    Sel sel;                                         // copy of the selection
    TypeInfo ty[kMaxTypes];
    __align__(16) unsigned char red[red_bytes<NW * 64>()];   // block_sum partials and totals
    double bcast[8];
};

// Returns the totals in LDS (valid until the next reduction's first
// barrier); block_sum copies them to every work-item.
template <int NT, int NV, typename T>
__device__ __forceinline__ const T* block_sum_lds(T (&v)[NV], unsigned char* red) {
    using G = RedGeom<NT, T>;
    static_assert(NV <= (sizeof(T) == 4 ? kRedNF : kRedND), "block_sum size");
    T* xbuf = reinterpret_cast<T*>(red);
    T* xtot = xbuf + NV * G::PS;
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
        if constexpr (G::Q == 4) v[i] = quad_sum(v[i]);
        if constexpr (G::Q == 16) v[i] = row_sum(v[i]);
        if constexpr (G::Q == 64) v[i] = wave_sum_last(v[i]);
    }
    constexpr int writer = G::Q == 64 ? 63 : 0;     // lane of each Q-group holding its sum
    if (tid % G::Q == writer) {
#pragma unroll
        for (int i = 0; i < NV; ++i) xbuf[i * G::PS + tid / G::Q] = v[i];
    }
    __syncthreads();
    // second stage: LPV lanes per value, so that all values fit one round
    // when 16 lanes each would need two.  Lane j of a value's group takes
    // the 16-byte slots j, j + LPV, ...: the group reads consecutive words.
    constexpr int LPV = (NV > NT / 16 && NV <= NT / 8) ? 8 : 16;
    for (int i0 = 0; i0 < NV; i0 += NT / LPV) {
        const int i = i0 + tid / LPV;
        const int j = tid % LPV;
        T acc = 0;
        if (i < NV) {
            const T* src = xbuf + i * G::PS;
            if constexpr (sizeof(T) == 4 && G::P % (4 * LPV) == 0) {
                // four running sums (one per component), so the chain of
                // dependent adds is short
                constexpr int E4 = G::P / (4 * LPV);
                const float4* s4 = reinterpret_cast<const float4*>(src);
                float4 a4 = s4[j];
#pragma unroll
                for (int e = 1; e < E4; ++e) {
                    const float4 q = s4[j + e * LPV];
                    a4.x += q.x;
                    a4.y += q.y;
                    a4.z += q.z;
                    a4.w += q.w;
                }
                acc = (a4.x + a4.y) + (a4.z + a4.w);
            } else {
                constexpr int E = (G::P + LPV - 1) / LPV;
#pragma unroll
                for (int e = 0; e < E; ++e)
                    if (j + e * LPV < G::P) acc += src[j + e * LPV];
            }
        }
        if constexpr (LPV == 16) acc = row_sum(acc);
        else acc = oct_sum(acc);
        if (i < NV && j == 0) xtot[i] = acc;
    }
    __syncthreads();
    return xtot;
}

template <int NT, int NV, typename T>
__device__ __forceinline__ void block_sum(T (&v)[NV], unsigned char* red) {
    const T* tot = block_sum_lds<NT, NV>(v, red);
#pragma unroll
    for (int i = 0; i < NV; ++i) v[i] = tot[i];
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

// The selection is read from an LDS copy: indexing the by-value kernel
// argument with a run-time type index would make the compiler copy the
// argument to private memory.  Thread 0 copies it with compile-time offsets.
__device__ __forceinline__ void copy_sel(const Sel& src, Sel& dst) {
    if (threadIdx.x == 0) {
        const int* a = reinterpret_cast<const int*>(&src);
        int* b = reinterpret_cast<int*>(&dst);
#pragma unroll
        for (int i = 0; i < (int)(sizeof(Sel) / sizeof(int)); ++i) b[i] = a[i];
    }
    __syncthreads();
}

// ------------------------------------------------------------- the solver
//
// Type indices are compile-time constants everywhere (loops over the types
// are unrolled to KMAX), so the selection is read straight from the kernel
// argument into scalar registers.

template <int NT, int APT, int KMAX>
struct Solver {
    static constexpr int NW = NT / 64;
    static constexpr int R1 = APT + 1;     // own rows: APT antennas + one type row
    const Sel& s;
    const TypeInfo* ty;
    unsigned char* red;          // block_sum buffers
    int N, K, n, tid;
    float4* rec;       // [N + K] {p_amp, p_phase, |g|^2 or |V|^2, scratch}
    double2* gd;       // [N] gains
    double2* vmd;      // [K] unique visibilities
    const void* vred;
    bool ci4;
    size_t vbase;
    const uint2* vl;   // the unit's V^reduced in LDS (raw 8-byte entries), or null
    // masked lattice: pair index table ([K][N], -1 where a pair does not
    // exist), antenna count and the first antenna (null / N / 0 otherwise)
    const int* pt;
    int n_live, ref0;
    // Only the one-antenna-per-work-item shapes (N <= 1024) take the LDS
    // copy: the larger grids' pairs do not fit beside the state, and their
    // register-bound kernels are left without the extra branches.
    static constexpr bool kVcache = APT == 1;
    // own antenna rows
    int a[APT], ax_[APT], ay_[APT];
    bool live[APT];
    unsigned m1[APT], m2[APT];   // bit t: pair (a, a - d_t) / (a + d_t, a) exists
    float gw[APT];               // own |g|^2 as published in the records
    // One antenna per work-item and few types: the pair weights and the
    // neighbours' record indices are kept in registers for a whole CG solve.
    static constexpr bool PW = APT == 1 && NT <= 512 && KMAX <= 8;
    float pw1[PW ? KMAX : 1], pw2[PW ? KMAX : 1];
    int nb1[PW ? KMAX : 1], nb2[PW ? KMAX : 1];
    bool own_t;
    // CG state of the own rows (index APT: the owned type row): solution,
    // residual, inverse diagonal, preconditioned residual
    float xa[R1], xp[R1], ra[R1], rp[R1], di[R1], ua[R1], up[R1];

    __device__ __forceinline__ Solver(const SolveLaunch& L, const TypeInfo* tyi, unsigned char* rd, unsigned char* lds,
                      int unit)
        : s(L.sel), ty(tyi), red(rd), vred(L.vred), ci4(L.ci4), vbase((size_t)unit * L.sel.P) {
        const bool vcache = L.vcache;
        N = s.N;
        K = s.K;
        n = s.n;
        tid = threadIdx.x;
        pt = L.mt.pidx;
        n_live = pt ? L.mt.n_live : N;
        ref0 = pt ? L.mt.ref0 : 0;
        const uint8_t* lv = L.mt.live;
        const SolveLayout Ly = solve_layout(s, vcache);
        rec = reinterpret_cast<float4*>(lds + Ly.rec);
        gd = reinterpret_cast<double2*>(lds + Ly.gd);
        vmd = reinterpret_cast<double2*>(lds + Ly.vmd);
        vl = nullptr;
        if (kVcache && vcache) {
            // one coalesced pass (published by a barrier before first use)
            uint2* dst = reinterpret_cast<uint2*>(lds + Ly.vr);
            const uint2* src = reinterpret_cast<const uint2*>(vred) + vbase;
            for (int b = tid; b < s.P; b += NT) dst[b] = src[b];
            vl = dst;
        }
        own_t = tid < K;
        if (own_t) rec[N + tid].w = __int_as_float(ty[tid].dxy);
#pragma unroll
        for (int k = 0; k < APT; ++k) {
            a[k] = tid + k * NT;
            // a grid point of a masked lattice without an antenna is no
            // unknown: it has no pairs, gain 0 and a zero record (which the
            // missing pairs of its neighbours read with weight 0)
            live[k] = a[k] < N && (!pt || lv[a[k]]);
            if (pt && a[k] < N && !live[k]) {
                rec[a[k]] = make_float4(0.f, 0.f, 0.f, 0.f);
                gd[a[k]] = make_double2(0.0, 0.0);
            }
            m1[k] = m2[k] = 0u;
            gw[k] = 0.f;
            ax_[k] = a[k] % n;
            ay_[k] = a[k] / n;
#pragma unroll
            for (int t = 0; t < KMAX; ++t) {
                if (t >= K || !live[k]) continue;
                const int dx = ty[t].dx, dy = ty[t].dy;
                const int jx = ax_[k] - dx, jy = ay_[k] - dy, ix = ax_[k] + dx, iy = ay_[k] + dy;
                if (jx >= 0 && jx < n && jy >= 0 && jy < n && (!pt || lv[jy * n + jx])) m1[k] |= 1u << t;
                if (ix >= 0 && ix < n && iy >= 0 && iy < n && (!pt || lv[iy * n + ix])) m2[k] |= 1u << t;
            }
        }
    }

    __device__ __forceinline__ bool mine(int k) const { return k < APT ? live[k] : own_t; }
    __device__ __forceinline__ int dxy(int t) const { return ty[t].dxy; }
    // pair (a, a - d_t) / (a + d_t, a) of own antenna k: affine in (x, y)
    // on a full grid, from the table on a masked lattice (MK)
    template <bool MK>
    __device__ __forceinline__ int b1v(int t, int k) const {
        if constexpr (MK) return pt[(size_t)t * N + a[k]];
        else return ty[t].c1 + ay_[k] * ty[t].w + ax_[k];
    }
    template <bool MK>
    __device__ __forceinline__ int b2v(int t, int k) const {
        if constexpr (MK) return pt[(size_t)t * N + a[k] + ty[t].dxy];
        else return ty[t].c2 + ay_[k] * ty[t].w + ax_[k];
    }
    __device__ __forceinline__ int b1(int t, int k) const { return pt ? b1v<true>(t, k) : b1v<false>(t, k); }
    __device__ __forceinline__ int b2(int t, int k) const { return pt ? b2v<true>(t, k) : b2v<false>(t, k); }
    __device__ __forceinline__ int ax(int k) const { return ax_[k]; }
    __device__ __forceinline__ int ay(int k) const { return ay_[k]; }

    // V^reduced of the unit's pair b, from the LDS copy when there is one
    __device__ __forceinline__ float2 vr32(int b) const {
        if (kVcache && vl) {
            const uint2 q = vl[b];
            return ci4 ? make_float2((float)(int)q.x, (float)(int)q.y)
                       : make_float2(__int_as_float((int)q.x), __int_as_float((int)q.y));
        }
        return load_vred(vred, ci4, vbase + b);
    }
    __device__ __forceinline__ double2 vr64(int b) const {
        if (kVcache && vl) {
            const uint2 q = vl[b];
            return ci4 ? make_double2((double)(int)q.x, (double)(int)q.y)
                       : make_double2(__int_as_float((int)q.x), __int_as_float((int)q.y));
        }
        return load_vred_d(vred, ci4, vbase + b);
    }
    // the same with the source fixed at compile time (VM bit 0: 4-bit sums,
    // bit 1: the LDS copy), for loops that must stay free of branches
    template <int VM>
    __device__ __forceinline__ double2 vr64v(int b) const {
        if constexpr ((VM & 2) != 0 && (VM & 4) == 0) {
            const uint2 q = vl[b];
            if constexpr ((VM & 1) != 0) return make_double2((double)(int)q.x, (double)(int)q.y);
            else return make_double2(__int_as_float((int)q.x), __int_as_float((int)q.y));
        } else {
            if constexpr ((VM & 1) != 0) {
                const int2 q = reinterpret_cast<const int2*>(vred)[vbase + b];
                return make_double2((double)q.x, (double)q.y);
            } else {
                const float2 f = reinterpret_cast<const float2*>(vred)[vbase + b];
                return make_double2(f.x, f.y);
            }
        }
    }

    // ---- residual pass: the right-hand sides ra, rp (J^H r split into its
    // amplitude and phase parts, scaled to unit norm; the scale is
    // returned), the inverse diagonal di of J^H J, and the weights of the
    // records.  FP64 throughout.  Each work-item recomputes the residuals
    // of its antennas' pairs; type rows are block sums over the pairs (each
    // pair counted at its first antenna), up to kChunk types at a time.
    __device__ __forceinline__ double residuals() {
        // one straight-line instance per V^reduced source (VM bit 2: the
        // masked lattice's pair table)
        if (pt) return ci4 ? residuals_v<5>() : residuals_v<4>();
        if constexpr (kVcache) {
            if (vl) return ci4 ? residuals_v<3>() : residuals_v<2>();
        }
        return ci4 ? residuals_v<1>() : residuals_v<0>();
    }

    template <int VM>
    __device__ __forceinline__ double residuals_v() {
        double rA[R1], rP[R1];
        float dd[R1];
#pragma unroll
        for (int k = 0; k < R1; ++k) {
            rA[k] = rP[k] = 0.0;
            dd[k] = 0.f;
        }
        double nrm = 0.0;
        constexpr int KC = KMAX < kChunk ? KMAX : kChunk;   // types per reduction
#pragma unroll
        for (int c0 = 0; c0 < KMAX; c0 += KC) {
            if (c0 >= K) break;
            double tq[3 * KC + 1];
#pragma unroll
            for (int i = 0; i < 3 * KC; ++i) tq[i] = 0.0;
#pragma unroll
            for (int tt = 0; tt < KC; ++tt) {
                const int t = c0 + tt;
                if (t >= K) break;
                const double2 vt = vmd[t];
                // e = 0: pair (a, a - d_t); e = 1: pair (a + d_t, a).  A
                // missing pair reads entry 0 and is dropped by a select.
                auto term = [&](int k, int e) {
                    const bool ok = live[k] && (((e ? m2[k] : m1[k]) >> t) & 1u);
                    const int i = ok ? (e ? a[k] + dxy(t) : a[k]) : 0;
                    const int j = ok ? i - dxy(t) : 0;
                    constexpr bool MK = (VM & 4) != 0;
                    const int b = ok ? (e ? b2v<MK>(t, k) : b1v<MK>(t, k)) : 0;
                    const double2 mm = dmul(dmulc(gd[i], gd[j]), vt);
                    const double2 q = dmulc(dsub(vr64v<VM>(b), mm), mm);
                    const double wb = ok ? dabs2(mm) : 0.0;
                    const double qx = ok ? q.x : 0.0, qy = ok ? q.y : 0.0;
                    rA[k] += qx;
                    rP[k] += e ? -qy : qy;
                    dd[k] += (float)wb;
                    if (!e) {
                        tq[tt] += qx;
                        tq[KC + tt] += qy;
                        tq[2 * KC + tt] += wb;
                    }
                };
                if constexpr (APT == 1) {
                    // straight-line, so every term's loads are in flight together
                    term(0, 0);
                    term(0, 1);
                } else {
                    // several antennas per work-item: a rolled loop that skips
                    // the missing pairs keeps registers and FP64 work down
#pragma unroll
                    for (int k = 0; k < APT; ++k) {
                        if (!live[k]) continue;
#pragma unroll 1
                        for (int e = 0; e < 2; ++e) {
                            if (!(((e ? m2[k] : m1[k]) >> t) & 1u)) continue;
                            term(k, e);
                        }
                    }
                }
            }
            // the antenna rows' |rhs|^2 rides on the last chunk's reduction,
            // when their right-hand sides are complete
            tq[3 * KC] = 0.0;
            if (c0 + KC >= K) {
#pragma unroll
                for (int k = 0; k < APT; ++k)
                    if (live[k]) tq[3 * KC] += rA[k] * rA[k] + rP[k] * rP[k];
            }
            block_sum<NT, 3 * KC + 1>(tq, red);
#pragma unroll
            for (int tt = 0; tt < KC; ++tt) {
                if (c0 + tt < K) nrm += tq[tt] * tq[tt] + tq[KC + tt] * tq[KC + tt];
                if (own_t && tid == c0 + tt) {
                    rA[APT] = tq[tt];
                    rP[APT] = tq[KC + tt];
                    dd[APT] = (float)tq[2 * KC + tt];
                }
            }
            if (c0 + KC >= K) nrm += tq[3 * KC];
        }
        const double scale = nrm > 0.0 ? sqrt(nrm) : 1.0;
        const double inv = 1.0 / scale;
#pragma unroll
        for (int k = 0; k < R1; ++k) {
            ra[k] = mine(k) ? (float)(rA[k] * inv) : 0.f;
            rp[k] = mine(k) ? (float)(rP[k] * inv) : 0.f;
            di[k] = dd[k] > 0.f ? 1.0f / dd[k] : 0.f;
        }
        return scale;
    }

    // |g|^2 of the own antennas and |V_t|^2 of the own type row into the
    // records, for the neighbours' matrix-vector products (published by the
    // barrier of the first reduction of the following CG solve).
    __device__ __forceinline__ void publish_weights(bool unit) {
#pragma unroll
        for (int k = 0; k < APT; ++k) {
            if (!live[k]) continue;
            gw[k] = unit ? 1.f : (float)dabs2(gd[a[k]]);
            rec[a[k]].z = gw[k];
        }
        if (own_t) rec[N + tid].z = unit ? 1.f : (float)dabs2(vmd[tid]);
    }

    // w = H u on the own rows of both systems, u read from the records, and
    // the dot products of one CG iteration, all in one block reduction:
    // the type rows' w are sums of their pairs' terms (each pair counted at
    // its first antenna); dots = {(r,u)_a, (r,u)_p, (u,w)_a, (u,w)_p}.
    // The type rows' part of (u,w), sum_t u_t w_t, is
    // summed term by term alongside (u_t times each pair term), so nothing
    // is read from the records after the reduction.
    // Pair weights |g_i|^2 |g_j|^2 |V_t|^2 and record indices of the own
    // antenna's pairs (zero weight and index 0 where a pair does not
    // exist), after the records' weights have been published.
    __device__ __forceinline__ void load_pair_weights() {
        if constexpr (PW) {
#pragma unroll
            for (int t = 0; t < KMAX; ++t) {
                pw1[t] = pw2[t] = 0.f;
                nb1[t] = nb2[t] = 0;
                if (t >= K) continue;
                const float vt = rec[N + t].z;
                const int dt = ty[t].dxy;
                const bool b1 = live[0] && ((m1[0] >> t) & 1u), b2 = live[0] && ((m2[0] >> t) & 1u);
                nb1[t] = b1 ? a[0] - dt : 0;
                nb2[t] = b2 ? a[0] + dt : 0;
                pw1[t] = b1 ? gw[0] * rec[nb1[t]].z * vt : 0.f;
                pw2[t] = b2 ? gw[0] * rec[nb2[t]].z * vt : 0.f;
            }
        }
    }

    __device__ __forceinline__ void matvec_dots(float (&wa)[R1], float (&wp)[R1], float (&dots)[4]) {
        constexpr int NV = 2 * KMAX + 4;
        float cs[NV];
#pragma unroll
        for (int i = 0; i < NV; ++i) cs[i] = 0.f;
#pragma unroll
        for (int k = 0; k < R1; ++k) wa[k] = wp[k] = 0.f;
        // Branch-free: a missing pair reads record 0 with weight 0; with
        // register weights the types past K also run, on the last type's
        // record with weight 0, so the loop is straight-line code, and all
        // the (u_amp, u_phase) reads are issued before any product.
        float2 qt[PW ? KMAX : 1], qj[PW ? KMAX : 1], qi[PW ? KMAX : 1];
        if constexpr (PW) {
            const float2* r2 = reinterpret_cast<const float2*>(rec);   // stride: 2 float2
#pragma unroll
            for (int t = 0; t < KMAX; ++t) {
                qt[t] = r2[2 * (N + (t >= K ? K - 1 : t))];
                qj[t] = r2[2 * nb1[t]];
                qi[t] = r2[2 * nb2[t]];
            }
        }
#pragma unroll
        for (int t = 0; t < KMAX; ++t) {
            if (!PW && t >= K) break;
            float4 rt;
            if constexpr (PW) rt = make_float4(qt[t].x, qt[t].y, 0.f, 0.f);
            else rt = rec[N + t];   // .z: |V_t|^2, .w: d_t
#pragma unroll
            for (int k = 0; k < APT; ++k) {
                float4 rj, ri;
                float w1, w2;
                if constexpr (PW) {
                    rj = make_float4(qj[t].x, qj[t].y, 0.f, 0.f);
                    ri = make_float4(qi[t].x, qi[t].y, 0.f, 0.f);
                    w1 = pw1[t];
                    w2 = pw2[t];
                } else {
                    const int dt = __float_as_int(rt.w);
                    const bool b1 = (m1[k] >> t) & 1u, b2 = (m2[k] >> t) & 1u;
                    rj = rec[b1 ? a[k] - dt : 0];
                    ri = rec[b2 ? a[k] + dt : 0];
                    w1 = b1 ? gw[k] * rj.z * rt.z : 0.f;
                    w2 = b2 ? gw[k] * ri.z * rt.z : 0.f;
                }
                // pair (a, j), j = a - d_t: a first
                const float eA = w1 * (ua[k] + rj.x + rt.x);
                const float eP = w1 * (up[k] - rj.y + rt.y);
                cs[t] += eA;
                cs[KMAX + t] += eP;
                cs[2 * KMAX + 2] += rt.x * eA;
                cs[2 * KMAX + 3] += rt.y * eP;
                // pair (i, a), i = a + d_t: a second
                wa[k] += eA + w2 * (ri.x + ua[k] + rt.x);
                wp[k] += eP - w2 * (ri.y - up[k] + rt.y);
            }
        }
#pragma unroll
        for (int k = 0; k < R1; ++k) {
            cs[2 * KMAX + 0] += ra[k] * ua[k];
            cs[2 * KMAX + 1] += rp[k] * up[k];
        }
#pragma unroll
        for (int k = 0; k < APT; ++k) {
            cs[2 * KMAX + 2] += ua[k] * wa[k];
            cs[2 * KMAX + 3] += up[k] * wp[k];
        }
        // every work-item needs the four dots; only the type-row owners
        // need their two type sums
        const float* tot = block_sum_lds<NT, NV>(cs, red);
#pragma unroll
        for (int i = 0; i < 4; ++i) dots[i] = tot[2 * KMAX + i];
        if (own_t) {
            wa[APT] = tot[tid];
            wp[APT] = tot[KMAX + tid];
        }
    }

    __device__ __forceinline__ void write_u() {
#pragma unroll
        for (int k = 0; k < APT; ++k) {
            if (!live[k]) continue;
            rec[a[k]].x = ua[k];
            rec[a[k]].y = up[k];
        }
        if (own_t) {
            rec[N + tid].x = ua[APT];
            rec[N + tid].y = up[APT];
        }
    }

    // Jacobi-preconditioned conjugate gradients on both systems from x = 0,
    // right-hand sides in ra / rp, inverse diagonal in di, weights in the
    // records.  The Chronopoulos-Gear arrangement: the recurrences
    // p = u + beta p and s = w + beta s (s = H p) need one matrix-vector
    // product (w = H u, u the preconditioned residual) and one reduction
    // per iteration.  Each system stops when its residual's preconditioned
    // norm (r, D^-1 r), a dot the iteration needs anyway, has fallen by
    // `tol`.  Returns the iterations, or -1 if a right-hand side is not
    // finite.
    __device__ __forceinline__ int pcg(int max_cg, float tol) {
        float pa[R1], pp[R1], sa[R1], sp[R1], wa[R1], wp[R1], dots[4];
#pragma unroll
        for (int k = 0; k < R1; ++k) {
            xa[k] = xp[k] = 0.f;
            ua[k] = ra[k] * di[k];
            up[k] = rp[k] * di[k];
        }
        write_u();
        __syncthreads();
        load_pair_weights();
        matvec_dots(wa, wp, dots);
        if (!(dots[0] == dots[0]) || !(dots[1] == dots[1]) || isinf(dots[0]) || isinf(dots[1])) return -1;
        const float stopa = tol * tol * dots[0], stopp = tol * tol * dots[1];
        bool done_a = !(dots[0] > 0.f), done_p = !(dots[1] > 0.f);
        float ga = dots[0], gp = dots[1];
        float ala = (!done_a && dots[2] > 0.f) ? ga / dots[2] : 0.f;
        float alp = (!done_p && dots[3] > 0.f) ? gp / dots[3] : 0.f;
#pragma unroll
        for (int k = 0; k < R1; ++k) {
            pa[k] = ua[k];
            pp[k] = up[k];
            sa[k] = wa[k];
            sp[k] = wp[k];
        }
        int it = 0;
        for (; it < max_cg && !(done_a && done_p); ++it) {
#pragma unroll
            for (int k = 0; k < R1; ++k) {
                xa[k] += ala * pa[k];
                xp[k] += alp * pp[k];
                ra[k] -= ala * sa[k];
                rp[k] -= alp * sp[k];
                ua[k] = ra[k] * di[k];
                up[k] = rp[k] * di[k];
            }
            write_u();
            __syncthreads();
            matvec_dots(wa, wp, dots);
            done_a = done_a || !(dots[0] > stopa);
            done_p = done_p || !(dots[1] > stopp);
            // scalars by hardware reciprocal (about 1 ulp): they only steer CG
            const float ba = ga > 0.f ? dots[0] * fast_rcp(ga) : 0.f;
            const float bp = gp > 0.f ? dots[1] * fast_rcp(gp) : 0.f;
            const float dena = dots[2] - (ala > 0.f ? ba * dots[0] * fast_rcp(ala) : 0.f);
            const float denp = dots[3] - (alp > 0.f ? bp * dots[1] * fast_rcp(alp) : 0.f);
            done_a = done_a || !(dena > 0.f);
            done_p = done_p || !(denp > 0.f);
            if (!done_a) {
                ala = dots[0] * fast_rcp(dena);
                ga = dots[0];
#pragma unroll
                for (int k = 0; k < R1; ++k) {
                    pa[k] = ua[k] + ba * pa[k];
                    sa[k] = wa[k] + ba * sa[k];
                }
            } else {
                ala = 0.f;
            }
            if (!done_p) {
                alp = dots[1] * fast_rcp(denp);
                gp = dots[1];
#pragma unroll
                for (int k = 0; k < R1; ++k) {
                    pp[k] = up[k] + bp * pp[k];
                    sp[k] = wp[k] + bp * sp[k];
                }
            } else {
                alp = 0.f;
            }
        }
        return it;
    }

    // V_t = mean over the group of V_b / (g_i conj(g_j)), in FP32.
    __device__ __forceinline__ void group_mean() {
        float sv[2 * KMAX];
#pragma unroll
        for (int i = 0; i < 2 * KMAX; ++i) sv[i] = 0.f;
#pragma unroll
        for (int t = 0; t < KMAX; ++t) {
            if (t >= K) break;
#pragma unroll
            for (int k = 0; k < APT; ++k) {
                if (!live[k] || !((m1[k] >> t) & 1u)) continue;
                const int b = b1(t, k);
                const float2 gg = cmulc(to_f(gd[a[k]]), to_f(gd[a[k] - dxy(t)]));
                const float2 q = cmulc(vr32(b), gg);
                const float inv = 1.0f / cabs2(gg);
                sv[t] += q.x * inv;
                sv[KMAX + t] += q.y * inv;
            }
        }
        block_sum<NT, 2 * KMAX>(sv, red);
#pragma unroll
        for (int t = 0; t < KMAX; ++t) {
            if (t >= K || !own_t || t != tid) continue;
            const float cnt = (float)ty[t].cnt;
            vmd[t] = to_d(make_float2(sv[t] / cnt, sv[KMAX + t] / cnt));
        }
        __syncthreads();
    }

    // Start, part 1: the logcal amplitude system (unit weights, right-hand
    // side sum of ln|V_b|) in ra / di, phase system empty.
    __device__ __forceinline__ void firstcal_rhs() {
        float tq[2 * KMAX];
#pragma unroll
        for (int i = 0; i < 2 * KMAX; ++i) tq[i] = 0.f;
        float rA[R1], dd[R1];
#pragma unroll
        for (int k = 0; k < R1; ++k) rA[k] = dd[k] = 0.f;
#pragma unroll
        for (int t = 0; t < KMAX; ++t) {
            if (t >= K) break;
#pragma unroll
            for (int k = 0; k < APT; ++k) {
                if (!live[k]) continue;
                if ((m1[k] >> t) & 1u) {
                    const int b = b1(t, k);
                    const float lv = 0.5f * logf(fmaxf(cabs2(vr32(b)), 1e-30f));
                    rA[k] += lv;
                    dd[k] += 1.f;
                    tq[t] += lv;
                    tq[KMAX + t] += 1.f;
                }
                if ((m2[k] >> t) & 1u) {
                    const int b = b2(t, k);
                    rA[k] += 0.5f * logf(fmaxf(cabs2(vr32(b)), 1e-30f));
                    dd[k] += 1.f;
                }
            }
        }
        block_sum<NT, 2 * KMAX>(tq, red);
#pragma unroll
        for (int t = 0; t < KMAX; ++t) {
            if (t >= K || !own_t || t != tid) continue;
            rA[APT] = tq[t];
            dd[APT] = tq[KMAX + t];
        }
#pragma unroll
        for (int k = 0; k < R1; ++k) {
            ra[k] = mine(k) ? rA[k] : 0.f;
            rp[k] = 0.f;
            di[k] = dd[k] > 0.f ? 1.0f / dd[k] : 0.f;
        }
        publish_weights(true);
    }

    // Start, part 2: amplitudes from the solved system, phases chained from
    // antenna (0,0) along the (1,0) group in the first row and the (0,1)
    // group up each column (each link's phase taken relative to the first
    // visibility of its group), into gd.
    __device__ __forceinline__ void firstcal_finish() {
        int off10 = 0, off01 = 0;
#pragma unroll
        for (int t = 0; t < KMAX; ++t) {
            if (t >= K) break;
            if (ty[t].dx == 1 && ty[t].dy == 0) off10 = ty[t].off;
            if (ty[t].dx == 0 && ty[t].dy == 1) off01 = ty[t].off;
        }
        const float2 v10 = vr32(off10);
        const float2 v01 = vr32(off01);
        const float psi10 = atan2f(v10.y, v10.x), psi01 = atan2f(v01.y, v01.x);
        const float2 r10 = make_float2(cosf(psi10), -sinf(psi10));
        const float2 r01 = make_float2(cosf(psi01), -sinf(psi01));
#pragma unroll
        for (int k = 0; k < APT; ++k) {
            if (!live[k]) continue;
            const int x = ax(k), y = ay(k);
            float inc = 0.f;
            if (y == 0 && x >= 1) {           // pair ((x,0), (x-1,0))
                const float2 v = cmul(vr32(off10 + (x - 1)), r10);
                inc = atan2f(v.y, v.x);
            } else if (y >= 1) {              // pair ((x,y), (x,y-1))
                const float2 v = cmul(vr32(off01 + (y - 1) * n + x), r01);
                inc = atan2f(v.y, v.x);
            }
            rec[a[k]].w = inc;
        }
        __syncthreads();
        if (tid == 0) {
            rec[0].w = 0.f;
            for (int x = 1; x < n; ++x) rec[x].w += rec[x - 1].w;
        }
        __syncthreads();
        if (tid < n) {
            for (int y = 1; y < n; ++y) rec[y * n + tid].w += rec[(y - 1) * n + tid].w;
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < APT; ++k) {
            if (!live[k]) continue;
            const float amp = expf(xa[k]);
            float sn, cs;
            sincosf(rec[a[k]].w, &sn, &cs);
            gd[a[k]] = to_d(make_float2(amp * cs, amp * sn));
        }
        __syncthreads();
    }

    // g <- g e^{eta}, V <- V e^{zeta} with (eta, zeta) = xscale * x, in
    // FP64.  The factor is formed as 1 + (small part), the small parts
    // (expm1 of the log-amplitude step, cos - 1 and sin of the phase step)
    // in FP32 to full relative precision, so the update keeps FP64 accuracy
    // however small the step.  Returns the rms step; the reduction's barrier
    // publishes g and V.
    __device__ __forceinline__ float update(double xscale) {
        float e2[1] = {0.f};
#pragma unroll
        for (int k = 0; k < R1; ++k) {
            if (!mine(k)) continue;
            const float ea = (float)(xa[k] * xscale), ep = (float)(xp[k] * xscale);
            e2[0] += ea * ea + ep * ep;
            const float sh = sinf(0.5f * ep);
            const double da = (double)expm1f(ea);
            const double dc = -2.0 * (double)(sh * sh);      // cos(ep) - 1
            const double sp = (double)sinf(ep);
            const double fr = (1.0 + da) * (1.0 + dc), fi = (1.0 + da) * sp;
            const double2 f = make_double2(fr, fi);
            if (k < APT) gd[a[k]] = dmul(gd[a[k]], f);
            else vmd[tid] = dmul(vmd[tid], f);
        }
        block_sum<NT, 1>(e2, red);
        return sqrtf(e2[0] / (float)(n_live + K));
    }
};

// The whole solve of one unit by one workgroup of NT work-items.
template <int NT, int APT, int KMAX>
__device__ __forceinline__ void solve_unit(const SolveLaunch& L, Shared<NT / 64>& sh, unsigned char* lds, int unit) {
    constexpr int NW = NT / 64;
    const Sel& s = L.sel;
    const SolveOpts op = L.o;
    if (threadIdx.x == 0) {
#pragma unroll
        for (int t = 0; t < KMAX; ++t) {
            if (t >= s.K) break;
            const int dx = s.dx[t], dy = s.dy[t], w = s.n - (dx < 0 ? -dx : dx);
            TypeInfo& T = sh.ty[t];
            T.dxy = dy * s.n + dx;
            T.w = w;
            T.c1 = s.off[t] - dy * w - (dx > 0 ? dx : 0);
            T.c2 = s.off[t] + (dx < 0 ? dx : 0);
            T.dx = dx;
            T.dy = dy;
            T.off = s.off[t];
            T.cnt = s.off[t + 1] - s.off[t];
        }
    }
    __syncthreads();
    Solver<NT, APT, KMAX> S(L, sh.ty, sh.red, lds, unit);
    const int N = S.N, K = S.K, tid = S.tid;
    __syncthreads();     // the LDS copy of V^reduced

    // ---- start: caller's gains, or the logcal solve (the first CG solve
    // of the loop below)
    bool start = !(op.init_mode == 1 && L.gains_in);
    if (!start) {
#pragma unroll
        for (int k = 0; k < APT; ++k)
            if (S.live[k]) S.gd[S.a[k]] = to_d(L.gains_in[(size_t)unit * N + S.a[k]]);
        __syncthreads();
        S.group_mean();
    }

    // ---- Gauss-Newton: FP32 steps while the rms step is above tol32 (at
    // most max_gn), then fp64_steps more
    int status = 0, steps = 0, n32 = 0;
    bool hi = false;
    int hi_left = op.fp64_steps;
    while (true) {
        double xscale = 1.0;
        if (start) {
            S.firstcal_rhs();
        } else {
            if (hi && hi_left <= 0) break;
            xscale = S.residuals();
            S.publish_weights(false);
        }
        // refinement steps start within about cg_tol of the solution, so
        // their normal equations need only sqrt(cg_tol)
        const int it = S.pcg(op.max_cg, start ? 1e-3f : (hi ? sqrtf(op.cg_tol) : op.cg_tol));
        if (start) {
            S.firstcal_finish();
            S.group_mean();
            start = false;
            continue;
        }
        if (it < 0) {           // non-finite data
            status = 2;
            break;
        }
        const float rms = S.update(xscale);
        ++steps;
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
            }
        }
    }

    // ---- degeneracies (FP64)
    if (op.degen_mode == 1 && L.gains_ref) {
        // match the mean log-amplitude and a phase plane to the reference
        double v9[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
#pragma unroll
        for (int k = 0; k < APT; ++k) {
            if (!S.live[k]) continue;
            const double2 gg = S.gd[S.a[k]];
            const double2 gr = to_d(L.gains_ref[(size_t)unit * N + S.a[k]]);
            const double2 q = dmulc(gg, gr);
            const double ph = atan2(q.y, q.x);
            const double x = S.ax(k), y = S.ay(k);
            v9[0] += 0.5 * log(dabs2(gg)) - 0.5 * log(dabs2(gr));
            v9[1] += ph;
            v9[2] += ph * x;
            v9[3] += ph * y;
            v9[4] += x;
            v9[5] += y;
            v9[6] += x * x;
            v9[7] += x * y;
            v9[8] += y * y;
        }
        block_sum<NT, 9>(v9, sh.red);
        if (tid == 0) {
            // [N  Sx  Sy ; Sx Sxx Sxy ; Sy Sxy Syy] c = [S, Sx, Sy] by Cramer's rule
            const double a00 = S.n_live, a01 = v9[4], a02 = v9[5], a11 = v9[6], a12 = v9[7], a22 = v9[8];
            const double det = a00 * (a11 * a22 - a12 * a12) - a01 * (a01 * a22 - a12 * a02) +
                               a02 * (a01 * a12 - a11 * a02);
            const double b0 = v9[1], b1 = v9[2], b2 = v9[3];
            const double c0 = (b0 * (a11 * a22 - a12 * a12) - a01 * (b1 * a22 - a12 * b2) +
                               a02 * (b1 * a12 - a11 * b2)) / det;
            const double c1 = (a00 * (b1 * a22 - a12 * b2) - b0 * (a01 * a22 - a12 * a02) +
                               a02 * (a01 * b2 - b1 * a02)) / det;
            const double c2 = (a00 * (a11 * b2 - b1 * a12) - a01 * (a01 * b2 - b1 * a02) +
                               b0 * (a01 * a12 - a11 * a02)) / det;
            sh.bcast[0] = exp(v9[0] / S.n_live);
            sh.bcast[1] = c0;
            sh.bcast[2] = c1;
            sh.bcast[3] = c2;
        }
    } else {
        // sum ln|g| = 0; the first antenna and its +x and +y neighbours
        // real ((0,0), (1,0) and (0,1) on a full grid)
        double v1[1] = {0.0};
#pragma unroll
        for (int k = 0; k < APT; ++k)
            if (S.live[k]) v1[0] += 0.5 * log(dabs2(S.gd[S.a[k]]));
        block_sum<NT, 1>(v1, sh.red);
        if (tid == 0) {
            const int r0 = S.ref0;
            const double2 g0 = S.gd[r0], g1 = S.gd[r0 + 1], gn = S.gd[r0 + s.n];
            const double2 qx = dmulc(g1, g0), qy = dmulc(gn, g0);
            sh.bcast[0] = exp(v1[0] / S.n_live);
            // the plane c0 + kx x + ky y through the references
            sh.bcast[2] = atan2(qx.y, qx.x);
            sh.bcast[3] = atan2(qy.y, qy.x);
            sh.bcast[1] = atan2(g0.y, g0.x) - sh.bcast[2] * (r0 % s.n) - sh.bcast[3] * (r0 / s.n);
        }
    }
    __syncthreads();
    {
        const double lam = sh.bcast[0], c0 = sh.bcast[1], kx = sh.bcast[2], ky = sh.bcast[3];
#pragma unroll
        for (int k = 0; k < APT; ++k) {
            if (!S.live[k]) continue;
            double sn, cs;
            sincos(-(c0 + kx * S.ax(k) + ky * S.ay(k)), &sn, &cs);
            const double2 gg = S.gd[S.a[k]];
            S.gd[S.a[k]] = make_double2((gg.x * cs - gg.y * sn) / lam, (gg.x * sn + gg.y * cs) / lam);
        }
#pragma unroll
        for (int t = 0; t < KMAX; ++t) {
            if (t >= K || !S.own_t || t != tid) continue;
            double sn, cs;
            sincos(kx * sh.ty[t].dx + ky * sh.ty[t].dy, &sn, &cs);
            const double2 v = S.vmd[t];
            const double l2 = lam * lam;
            S.vmd[t] = make_double2((v.x * cs - v.y * sn) * l2, (v.x * sn + v.y * cs) * l2);
        }
    }
    __syncthreads();

    // ---- chi^2 (FP64) and outputs
    double c1[1] = {0.0};
#pragma unroll
    for (int t = 0; t < KMAX; ++t) {
        if (t >= K) break;
#pragma unroll
        for (int k = 0; k < APT; ++k) {
            if (!S.live[k] || !((S.m1[k] >> t) & 1u)) continue;
            const int b = S.b1(t, k);
            const double2 mm = dmul(dmulc(S.gd[S.a[k]], S.gd[S.a[k] - S.dxy(t)]), S.vmd[t]);
            c1[0] += dabs2(dsub(S.vr64(b), mm));
        }
    }
    block_sum<NT, 1>(c1, sh.red);
#pragma unroll
    for (int k = 0; k < APT; ++k) {
        if (S.live[k]) L.gains_out[(size_t)unit * N + S.a[k]] = to_f(S.gd[S.a[k]]);
        else if (S.a[k] < N) L.gains_out[(size_t)unit * N + S.a[k]] = make_float2(0.f, 0.f);
    }
    if (S.own_t) L.vmodel[(size_t)unit * K + tid] = to_f(S.vmd[tid]);
    if (tid == 0) {
        const bool fin = c1[0] == c1[0] && !isinf(c1[0]);
        L.chisq[unit] = (float)c1[0];
        L.niter[unit] = steps;
        L.status[unit] = fin ? status : 2;
    }
#ifndef RRC_HOST_EMU
    if (L.stamps) {
        // completion time of this unit's solve (every work-item's outputs
        // are written before the barrier)
        __syncthreads();
        if (tid == 0) unit_done_stamp(L.stamps, unit);
    }
#endif
}

#ifndef RRC_HOST_EMU
template <int NT, int APT, int KMAX>
__global__ __launch_bounds__(NT) void k_solve(SolveLaunch L) {
    extern __shared__ __align__(16) unsigned char ssm[];
    __shared__ Shared<NT / 64> sh;
    solve_unit<NT, APT, KMAX>(L, sh, ssm, blockIdx.x);
}

// PREP: only raise the instantiation's dynamic-LDS limit to a whole CU's
// (a host runtime call, made once per plan before any launch, so that the
// launch path itself -- which a caller may capture into a graph -- makes
// kernel launches only); otherwise launch.
template <int NT, int APT, int KMAX>
static hipError_t launch_solve_k(const SolveLaunch& L, hipStream_t st, bool prep) {
    auto kern = k_solve<NT, APT, KMAX>;
    const size_t whole = kLdsPerCu - sizeof(Shared<NT / 64>);
    if (prep)
        return hipFuncSetAttribute(reinterpret_cast<const void*>(kern),
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)whole);
    size_t lds = L.lds_bytes;
    // a unit per CU at most: claim the CU's whole LDS, so that kernels
    // running beside the solve (the pipelined FFT) take other CUs instead of
    // sharing this latency-bound workgroup's SIMDs
    if (L.exclusive && whole > lds) lds = whole;
    hipLaunchKernelGGL(kern, dim3(L.n_units), dim3(NT), lds, st, L);
    return hipGetLastError();
}

template <int NT, int APT>
static hipError_t launch_solve_shape(const SolveLaunch& L, hipStream_t st, bool prep) {
    if (L.sel.K <= 6) return launch_solve_k<NT, APT, 6>(L, st, prep);
    if (L.sel.K <= 8) return launch_solve_k<NT, APT, 8>(L, st, prep);
    if (L.sel.K <= 10) return launch_solve_k<NT, APT, 10>(L, st, prep);
    return launch_solve_k<NT, APT, kMaxTypes>(L, st, prep);
}

static hipError_t solve_dispatch(const SolveLaunch& L, hipStream_t st, bool prep) {
    const int N = L.sel.N;
    if (L.sel.K < 1 || L.sel.K > kMaxTypes || L.sel.K > solve_threads_for(N)) return hipErrorInvalidValue;
    if (N <= 256) return launch_solve_shape<256, 1>(L, st, prep);
    if (N <= 512) return launch_solve_shape<512, 1>(L, st, prep);
    // larger grids: 512 work-items (256 VGPRs each) rather than 1024 (128),
    // with as few antennas per work-item as cover the grid (at 48 x 48, five
    // instead of eight take the solve from 3.5 to 1.2 ms: no spills; at
    // 32 x 32, two per work-item instead of 1024 work-items of one, which
    // spilled, 0.455 -> 0.413 ms)
    if (N <= 1024) return launch_solve_shape<512, 2>(L, st, prep);
    if (N <= 2048) return launch_solve_shape<512, 4>(L, st, prep);
    if (N <= 2560) return launch_solve_shape<512, 5>(L, st, prep);
    if (N <= 4096) return launch_solve_shape<512, 8>(L, st, prep);
    return hipErrorInvalidValue;
}

hipError_t prepare_solve(const SolveLaunch& L) { return solve_dispatch(L, nullptr, true); }

hipError_t launch_solve(const SolveLaunch& L, hipStream_t st) { return solve_dispatch(L, st, false); }

// --------------------------------------------------- chi^2 and its adjoint
//
// One workgroup of 256 work-items per unit.  Forward: sum_b |r_b|^2 in
// FP64 over FP32 products.  Adjoint (a6): antenna-centric gathers over the
// (at most 2K) incident pairs with r_b recomputed on the fly; type rows
// summed by one wave per type over the type's pairs.

constexpr int kCThreads = 256;

template <int APT, bool ADJ>
__global__ __launch_bounds__(kCThreads) void k_chisq(ChisqLaunch L) {
    __shared__ Sel ssel;
    __shared__ __align__(16) unsigned char sred[(RedGeom<kCThreads, double>::PS + 1) * 8];
    copy_sel(L.sel, ssel);
    const Sel& s = ssel;
    const int unit = blockIdx.x;
    const int N = s.N, K = s.K, n = s.n;
    const float2* g = L.g + (size_t)unit * N;
    const float2* vm = L.vm + (size_t)unit * K;
    const float2* vr = L.vred + (size_t)unit * s.P;
    if constexpr (!ADJ) {
        double c1[1] = {0.0};
        for (int t = 0; t < K; ++t) {
            const int dxy = s.dy[t] * n + s.dx[t];
#pragma unroll
            for (int k = 0; k < APT; ++k) {
                const int a = threadIdx.x + k * kCThreads;
                if (a >= N) continue;
                const int b = pair_as_first(s, t, a % n, a / n);
                if (b < 0) continue;
                const float2 r = csub(vr[b], cmul(cmulc(g[a], g[a - dxy]), vm[t]));
                c1[0] += (double)cabs2(r);
            }
        }
        block_sum<kCThreads, 1>(c1, sred);
        if (threadIdx.x == 0) L.chisq[unit] = (float)c1[0];
    } else {
        // antenna rows
#pragma unroll
        for (int k = 0; k < APT; ++k) {
            const int a = threadIdx.x + k * kCThreads;
            if (a >= N) continue;
            const int x = a % n, y = a / n;
            float2 gr = make_float2(0.f, 0.f);
            float dg = 0.f;
            for (int t = 0; t < K; ++t) {
                const int dxy = s.dy[t] * n + s.dx[t];
                const int b1 = pair_as_first(s, t, x, y);
                if (b1 >= 0) {   // pair (a, j): - r_b g_j conj(V_t)
                    const int j = a - dxy;
                    const float2 c = cmulc(g[j], vm[t]);
                    const float2 r = csub(vr[b1], cmul(cmulc(g[a], g[j]), vm[t]));
                    gr = csub(gr, cmul(r, c));
                    dg += cabs2(c);
                }
                const int b2 = pair_as_second(s, t, x, y);
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
        // type rows
        const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
        for (int t = wave; t < K; t += kCThreads / 64) {
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
    if (adj) hipLaunchKernelGGL((k_chisq<APT, true>), dim3(L.n_units), dim3(kCThreads), 0, st, L);
    else hipLaunchKernelGGL((k_chisq<APT, false>), dim3(L.n_units), dim3(kCThreads), 0, st, L);
    return hipGetLastError();
}

hipError_t launch_chisq(const ChisqLaunch& L, hipStream_t st, bool adjoint) {
    const int apt = (L.sel.N + kCThreads - 1) / kCThreads;
    if (apt <= 1) return launch_chisq_apt<1>(L, st, adjoint);
    if (apt <= 4) return launch_chisq_apt<4>(L, st, adjoint);
    if (apt <= 16) return launch_chisq_apt<16>(L, st, adjoint);
    return hipErrorInvalidValue;
}
#endif  // RRC_HOST_EMU

}  // namespace rrc
