// Redundant calibration by damped simultaneous per-parameter updates: the
// omnical iteration the paper's simulations use (Sec. 3: damping 0.3,
// convergence 1e-10; the update rule itself is cited there, not written).
// Holding every other parameter fixed, chi^2 of eq. redchi is an exact
// quadratic in one g_i or one V_alpha (no pair has i = j), whose minimiser is
//     g_i'     = [ sum_{(i,j)} V_b g_j conj(V_a) + sum_{(k,i)} conj(V_b) g_k V_b' ]
//                / [ sum |g_j V_a|^2 + sum |g_k V_b'|^2 ],
//     V_alpha' = sum_{b in alpha} V_b conj(g_i) g_j / sum |g_i g_j|^2;
// all parameters move together, x <- x + 0.3 (x' - x), until the relative
// change ||x_new - x|| / ||x_new|| falls below the tolerance.
//
// One workgroup per unit, the unit's gains and model visibilities in LDS
// (FP32), V^reduced read from HBM.  The type list is either the plan's
// selection or every canonical type of the grid in V^unique's lag order
// (the full pair set that low-cadence calibration solves, Sec. 4), whose
// pair offsets the workgroup derives at start.  Each call runs up to
// max_iter iterations and adds them to niter: one call per iteration with
// the change read back on the host is the plain per-channel form, one call
// with many iterations converges on the device.  The finishing call fixes
// the degeneracies (sum ln|g| = 0; antennas (0,0), (1,0), (0,1) real,
// Sec. 5.2) and computes chi^2 in FP64.
#include "rrc_device.h"
#include "rrc_launch.h"

namespace rrc {

constexpr int kOThreads = 256;
constexpr int kOMaxAllGrid = 32;        // every-type lists up to 32 x 32 (1984 types)

__device__ __forceinline__ int o_count(int n, int dx, int dy) { return (n - (dx < 0 ? -dx : dx)) * (n - dy); }

// canonical type t of an n x n grid in lag order (dy ascending, then dx;
// dy = 0 starts at dx = 1)
__device__ __forceinline__ void o_lag(int n, int t, int& dx, int& dy) {
    if (t < n - 1) {
        dx = t + 1;
        dy = 0;
    } else {
        const int u = t - (n - 1);
        dy = 1 + u / (2 * n - 1);
        dx = u % (2 * n - 1) - (n - 1);
    }
}

template <typename T>
__device__ __forceinline__ T o_wave_sum(T v) {
    for (int o = 1; o < 64; o <<= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// sum over the workgroup, result to every work-item (two barriers)
template <typename T>
__device__ __forceinline__ T o_block_sum(T v, T* red) {
    v = o_wave_sum(v);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) red[wave] = v;
    __syncthreads();
    T s = 0;
    for (int w = 0; w < kOThreads / 64; ++w) s += red[w];
    return s;
}

__global__ __launch_bounds__(kOThreads) void k_omnical(OmniLaunch L) {
    extern __shared__ __align__(16) unsigned char osm[];
    __shared__ double dred[kOThreads / 64];
    __shared__ float fred[kOThreads / 64];
    const int n = L.n, N = n * n, K = L.K;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int unit = blockIdx.x;
    // LDS: type table (every-type lists only), gains, model visibilities
    int* tdx = reinterpret_cast<int*>(osm);
    int* tdy = tdx + K;
    int* toff = tdy + K;                                  // K + 1 entries
    float2* g = reinterpret_cast<float2*>(osm + L.lds_types);
    float2* vm = g + N;
    float2* gn = vm + K;                                  // the iteration's new values
    float2* vn = gn + N;

    // ---- type table
    if (L.all) {
        for (int t = tid; t < K; t += kOThreads) {
            int dx, dy;
            o_lag(n, t, dx, dy);
            tdx[t] = dx;
            tdy[t] = dy;
        }
        __syncthreads();
        if (tid == 0) {
            int acc = 0;
            for (int t = 0; t < K; ++t) {
                toff[t] = acc;
                acc += o_count(n, tdx[t], tdy[t]);
            }
            toff[K] = acc;
        }
        __syncthreads();
    }
    auto typ = [&](int t, int& dx, int& dy, int& off, int& cnt) {
        if (L.all) {
            dx = tdx[t];
            dy = tdy[t];
            off = toff[t];
            cnt = toff[t + 1] - off;
        } else {
            dx = L.sel.dx[t];
            dy = L.sel.dy[t];
            off = L.sel.off[t];
            cnt = L.sel.off[t + 1] - off;
        }
    };
    // A masked lattice (a hexagonal array on its grid): pairs come from the
    // tables, grid points without an antenna keep gain 0 and take no part,
    // and the references of the degeneracy fix are the first antenna and
    // its +x and +y neighbours.
    const bool masked = L.mt.pidx != nullptr;
    const int n_live = masked ? L.mt.n_live : N, ref0 = masked ? L.mt.ref0 : 0;
    auto alive = [&](int a) { return !masked || L.mt.live[a] != 0; };
    // first antenna of pair b of a type
    auto first_of = [&](int off, int b, int dx, int dy, int w) {
        return masked ? L.mt.pfirst[off + b] : (b / w + dy) * n + b % w + (dx > 0 ? dx : 0);
    };
    // V^reduced index of pair (a, a - d_t) (both on the grid), or -1
    auto pair_at = [&](int t, int off, int a, int jx, int jy, int w, int dx) {
        return masked ? L.mt.pidx[(size_t)t * N + a] : off + jy * w + (a % n) - (dx > 0 ? dx : 0);
    };
    // V^reduced: complex64, or raw int32 sums (4-bit plans) read as floats
    const float2* vrf = reinterpret_cast<const float2*>(L.vred) + (size_t)unit * L.P;
    const int2* vri = reinterpret_cast<const int2*>(L.vred) + (size_t)unit * L.P;
    auto vr_at = [&](int b) -> float2 {
        if (L.ci4) {
            const int2 v = vri[b];
            return make_float2((float)v.x, (float)v.y);
        }
        return vrf[b];
    };
    float2* gout = reinterpret_cast<float2*>(L.gains) + (size_t)unit * N;
    float2* vout = reinterpret_cast<float2*>(L.vmodel) + (size_t)unit * K;

    // ---- state: from gains_in (V from the group means), or continued
    if (L.gains_in) {
        for (int a = tid; a < N; a += kOThreads)
            g[a] = alive(a) ? L.gains_in[(size_t)unit * N + a] : make_float2(0.f, 0.f);
        __syncthreads();
        for (int t = wave; t < K; t += kOThreads / 64) {
            int dx, dy, off, cnt;
            typ(t, dx, dy, off, cnt);
            const int w = n - (dx < 0 ? -dx : dx);
            float sr = 0.f, si = 0.f;
            for (int b = lane; b < cnt; b += 64) {
                const int i = first_of(off, b, dx, dy, w), j = i - (dy * n + dx);
                const float2 gg = cmulc(g[i], g[j]);            // g_i conj(g_j)
                const float2 q = cmulc(vr_at(off + b), gg);        // V_b conj(g_i conj(g_j))
                const float d = cabs2(gg);
                sr += q.x / d;
                si += q.y / d;
            }
            sr = o_wave_sum(sr);
            si = o_wave_sum(si);
            if (lane == 0) vm[t] = make_float2(sr / cnt, si / cnt);
        }
    } else {
        for (int a = tid; a < N; a += kOThreads) g[a] = gout[a];
        for (int t = tid; t < K; t += kOThreads) vm[t] = vout[t];
    }
    __syncthreads();

    int it = 0, status = 1;
    float rel = 0.f;
    for (; it < L.max_iter; ++it) {
        // antennas: the minimiser of each single g_i
        for (int a = tid; a < N; a += kOThreads) {
            const int ax = a % n, ay = a / n;
            float2 num = make_float2(0.f, 0.f);
            float den = 0.f;
            for (int t = 0; t < K; ++t) {
                int dx, dy, off, cnt;
                typ(t, dx, dy, off, cnt);
                const int w = n - (dx < 0 ? -dx : dx);
                const int jx = ax - dx, jy = ay - dy;
                if (jx >= 0 && jx < n && jy >= 0) {          // (a, j): V_b g_j conj(V_t)
                    const int b = pair_at(t, off, a, jx, jy, w, dx);
                    if (b >= 0) {
                        const float2 c = cmulc(g[jy * n + jx], vm[t]);
                        num = cadd(num, cmul(vr_at(b), c));
                        den += cabs2(c);
                    }
                }
                const int ix = ax + dx, iy = ay + dy;
                if (ix >= 0 && ix < n && iy < n) {           // (i, a): conj(V_b) g_i V_t
                    const int b = pair_at(t, off, iy * n + ix, ax, ay, w, dx);
                    if (b >= 0) {
                        const float2 c = cmul(g[iy * n + ix], vm[t]);
                        num = cadd(num, cmul(cconj(vr_at(b)), c));
                        den += cabs2(c);
                    }
                }
            }
            // a grid point with no antenna has no pair: it keeps its gain (0)
            gn[a] = den > 0.f ? make_float2(num.x / den, num.y / den) : g[a];
        }
        // types: the minimiser of each single V_alpha
        for (int t = wave; t < K; t += kOThreads / 64) {
            int dx, dy, off, cnt;
            typ(t, dx, dy, off, cnt);
            const int w = n - (dx < 0 ? -dx : dx);
            float sr = 0.f, si = 0.f, sd = 0.f;
            for (int b = lane; b < cnt; b += 64) {
                const int i = first_of(off, b, dx, dy, w), j = i - (dy * n + dx);
                const float2 gg = cmulc(g[j], g[i]);            // conj(g_i) g_j
                const float2 q = cmul(vr_at(off + b), gg);
                sr += q.x;
                si += q.y;
                sd += cabs2(gg);
            }
            sr = o_wave_sum(sr);
            si = o_wave_sum(si);
            sd = o_wave_sum(sd);
            if (lane == 0) vn[t] = make_float2(sr / sd, si / sd);
        }
        __syncthreads();
        // damped simultaneous update and the relative change
        float dn = 0.f, xn = 0.f;
        for (int q = tid; q < N + K; q += kOThreads) {
            const float2 x0 = q < N ? g[q] : vm[q - N];
            const float2 x1 = q < N ? gn[q] : vn[q - N];
            const float2 d = make_float2(L.damping * (x1.x - x0.x), L.damping * (x1.y - x0.y));
            const float2 x = cadd(x0, d);
            if (q < N) g[q] = x;
            else vm[q - N] = x;
            dn += cabs2(d);
            xn += cabs2(x);
        }
        dn = o_block_sum(dn, fred);
        xn = o_block_sum(xn, fred);
        rel = sqrtf(dn / xn);
        if (!(rel == rel)) {
            status = 2;
            ++it;
            break;
        }
        if (rel < L.tol) {
            status = 0;
            ++it;
            break;
        }
    }
    __syncthreads();

    if (L.finish) {
        // degeneracies (FP64): sum ln|g| = 0 over the antennas; the first
        // antenna and its +x, +y neighbours real ((0,0), (1,0), (0,1) on a
        // full grid)
        double ls = 0.0;
        for (int a = tid; a < N; a += kOThreads)
            if (alive(a)) ls += 0.5 * log((double)cabs2(g[a]));
        ls = o_block_sum(ls, dred);
        const double lam = exp(ls / n_live);
        const double2 g0 = to_d(g[ref0]), g1 = to_d(g[ref0 + 1]), gy = to_d(g[ref0 + n]);
        const double2 qx = dmulc(g1, g0), qy = dmulc(gy, g0);
        const double c0 = atan2(g0.y, g0.x), kx = atan2(qx.y, qx.x), ky = atan2(qy.y, qy.x);
        const int x0 = ref0 % n, y0 = ref0 / n;
        __syncthreads();
        for (int a = tid; a < N; a += kOThreads) {
            double sn, cs;
            sincos(-(c0 + kx * (a % n - x0) + ky * (a / n - y0)), &sn, &cs);
            const double2 x = to_d(g[a]);
            g[a] = to_f(make_double2((x.x * cs - x.y * sn) / lam, (x.x * sn + x.y * cs) / lam));
        }
        for (int t = tid; t < K; t += kOThreads) {
            int dx, dy, off, cnt;
            typ(t, dx, dy, off, cnt);
            double sn, cs;
            sincos(kx * dx + ky * dy, &sn, &cs);
            const double2 v = to_d(vm[t]);
            vm[t] = to_f(make_double2((v.x * cs - v.y * sn) * lam * lam, (v.x * sn + v.y * cs) * lam * lam));
        }
        __syncthreads();
        // chi^2 (FP64 sum over the pairs)
        double c2 = 0.0;
        for (int t = wave; t < K; t += kOThreads / 64) {
            int dx, dy, off, cnt;
            typ(t, dx, dy, off, cnt);
            const int w = n - (dx < 0 ? -dx : dx);
            for (int b = lane; b < cnt; b += 64) {
                const int i = first_of(off, b, dx, dy, w), j = i - (dy * n + dx);
                const double2 m = dmul(dmulc(to_d(g[i]), to_d(g[j])), to_d(vm[t]));
                c2 += dabs2(dsub(to_d(vr_at(off + b)), m));
            }
        }
        c2 = o_block_sum(c2, dred);
        if (tid == 0) {
            L.chisq[unit] = (float)c2;
            L.status[unit] = (c2 == c2) ? status : 2;
        }
    }
    for (int a = tid; a < N; a += kOThreads) gout[a] = g[a];
    for (int t = tid; t < K; t += kOThreads) vout[t] = vm[t];
    if (tid == 0) {
        L.niter[unit] = (L.gains_in ? 0 : L.niter[unit]) + it;
        if (L.delta) L.delta[unit] = rel;
        if (!L.finish) L.status[unit] = status;
    }
}

int omnical_max_all_grid() { return kOMaxAllGrid; }

size_t omnical_lds_bytes(int n, int K, bool all) {
    const size_t types = all ? (size_t)(3 * K + 1) * 4 : 0;
    const size_t tpad = (types + 15) / 16 * 16;
    return tpad + (size_t)2 * (n * n + K) * 8;
}

hipError_t launch_omnical(const OmniLaunch& L, hipStream_t st) {
    if (L.all && L.n > kOMaxAllGrid) return hipErrorInvalidValue;
    const size_t lds = omnical_lds_bytes(L.n, L.K, L.all);
    hipLaunchKernelGGL(k_omnical, dim3(L.n_units), dim3(kOThreads), lds, st, L);
    return hipGetLastError();
}

}  // namespace rrc
