// The C-ABI of include/rrcal.h: plans, the subset selection rule, the
// degeneracy count, argument checking and kernel dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <string>
#include <mutex>
#include <new>
#include <vector>

#include "../../include/rrcal.h"
#include "rrc_launch.h"

using rrc::Sel;

struct rrc_plan {
    Sel sel;
    int M;
    int nlag;
    int U, T, dtype;
    rrc_solver_opts opts;
    // FFT-correlator
    int fft_tchunk, fft_nchunk;
    int fft_tchunk0;                 // the default chunk (the workspace is sized for it)
    int M_default = 0;               // the smallest size whose lags do not wrap (see plan_create)
    int M_alt = 0;                   // the next power of two when it differs, else 0
    // X-engine; 4-bit plans whose window cover an int8 matrix-core
    // instantiation holds use it (x_mf: its launch fields) unless the
    // caller selects the dot-product kernel
    int x_tchunk, x_nchunk, x_nablk, x_S, x_halo;
    bool x_mf_ok = false;
    int32_t x_kind = RRC_XENG_AUTO;
    rrc::XengLaunch x_mf{};
    // solver
    bool solve_vcache;
    size_t solve_lds_bytes;
    // workspace layout
    size_t off_fft, off_x, off_gcopy, ws_bytes;
    size_t off_hinv = 0;             // 1/g table of the M = 96 kernel
    // pipelined run: the FFT-correlator forked after the X-engine (default)
    // or before it (RRC_ORDER_FFT_FIRST)
    int32_t order = RRC_ORDER_XENG_FIRST;
    // device resources, made by prepare() on the first device call (the
    // device current then): the fork/join stream and events of the
    // pipelined run (default priority), the CU count, the solve's LDS limit
    bool prepared = false;
    int device = -1;
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    int cu_count = 0;
    // rrc_run_static: the static scratch's address on this device
    void* scratch = nullptr;
    // units launched concurrently with this plan's (a batch sets the sum of
    // its plans'); the solve claims whole CUs only when they all fit
    long concurrent_units = 0;
    // masked lattice (rrc_plan_create_masked): the mask as bits, the antenna
    // count, the first antenna in raster order, and the workspace offsets of
    // the tables rebuilt from the mask by each device call
    bool masked = false;
    uint32_t mask_bits[rrc::kMaskWords] = {0};
    int n_live = 0, ref0 = 0;
    size_t off_live = 0, off_pidx = 0, off_pfirst = 0, off_nd = 0;
};

struct rrc_batch {
    std::vector<rrc_plan*> plans;
    uint32_t flags = 0;
    bool prepared = false;
    std::vector<hipStream_t> branch;           // one per plan
    std::vector<hipEvent_t> ev_done;           // one per plan
    hipEvent_t ev_start = nullptr;
};

namespace {

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

struct Type {
    int dx, dy;
};

// |d|^2 of a lattice displacement: square basis, or the hexagonal lattice's
// (1, 0), (1/2, sqrt3/2) basis (|d|^2 = dx^2 + dx dy + dy^2)
int metric_len2(int dx, int dy, int metric) {
    return metric == RRC_METRIC_HEX ? dx * dx + dx * dy + dy * dy : dx * dx + dy * dy;
}

// Canonical types of an n x n grid sorted by (|d|^2, dy, dx).
std::vector<Type> sorted_types(int n, int metric = RRC_METRIC_SQUARE) {
    std::vector<Type> t;
    for (int dy = 0; dy < n; ++dy)
        for (int dx = -(n - 1); dx < n; ++dx)
            if (dy > 0 || dx > 0) t.push_back({dx, dy});
    std::sort(t.begin(), t.end(), [metric](const Type& a, const Type& b) {
        const int la = metric_len2(a.dx, a.dy, metric), lb = metric_len2(b.dx, b.dy, metric);
        if (la != lb) return la < lb;
        if (a.dy != b.dy) return a.dy < b.dy;
        return a.dx < b.dx;
    });
    return t;
}

bool bit_of(const uint32_t* bits, int a) { return bits == nullptr || ((bits[a >> 5] >> (a & 31)) & 1u); }

// Pairs of type (dx, dy) whose antennas both exist (bits == nullptr: all).
long group_size_masked(int n, const uint32_t* bits, int dx, int dy) {
    if (!bits) return (long)(n - std::abs(dx)) * (n - std::abs(dy));
    long c = 0;
    for (int y = std::max(0, dy); y < n; ++y)
        for (int x = std::max(0, dx); x < n + std::min(0, dx); ++x)
            c += bit_of(bits, y * n + x) && bit_of(bits, (y - dy) * n + (x - dx));
    return c;
}

void pack_mask(int n, const uint8_t* mask, uint32_t* bits) {
    std::memset(bits, 0, sizeof(uint32_t) * rrc::kMaskWords);
    for (int a = 0; a < n * n; ++a)
        if (mask[a]) bits[a >> 5] |= 1u << (a & 31);
}

int group_size(int n, int dx, int dy) { return (n - std::abs(dx)) * (n - std::abs(dy)); }

bool valid_type(int n, int dx, int dy) {
    if (std::abs(dx) >= n || dy < 0 || dy >= n) return false;
    return dy > 0 || dx > 0;
}

// Null-space dimension of the normal matrix of a system whose rows are
// e_i + s e_j + e_{N+t} (s = +1 amplitude, -1 phase) over all selected
// pairs.  The matrix is assembled in skyline (profile) storage with the
// antennas in raster order and the K type unknowns last, and factored as
// L D L^T without pivoting; a positive semi-definite matrix meets a zero
// pivot exactly on each null direction, counted against a relative
// tolerance.
int normal_nullity(int n, const std::vector<Type>& sel, int sign, const uint32_t* bits = nullptr) {
    const int N = n * n, K = (int)sel.size(), V = N + K;
    int bw = 0;
    for (const Type& t : sel) bw = std::max(bw, t.dy * n + std::abs(t.dx));
    std::vector<int> first(V);
    for (int r = 0; r < V; ++r) first[r] = r < N ? std::max(0, r - bw) : 0;
    std::vector<size_t> start(V + 1, 0);
    for (int r = 0; r < V; ++r) start[r + 1] = start[r] + (size_t)(r - first[r] + 1);
    std::vector<double> A(start[V], 0.0);
    auto at = [&](int r, int c) -> double& {      // c <= r, c >= first[r]
        return A[start[r] + (size_t)(c - first[r])];
    };
    for (int t = 0; t < K; ++t) {
        const int dx = sel[t].dx, dy = sel[t].dy;
        for (int y = 0; y < n; ++y)
            for (int x = 0; x < n; ++x) {
                const int jx = x - dx, jy = y - dy;
                if (jx < 0 || jx >= n || jy < 0 || jy >= n) continue;
                const int i = y * n + x, j = jy * n + jx;
                if (!bit_of(bits, i) || !bit_of(bits, j)) continue;
                const int idx[3] = {i, j, N + t};
                const double cf[3] = {1.0, (double)sign, 1.0};
                for (int p = 0; p < 3; ++p)
                    for (int q = 0; q <= p; ++q) {
                        int r = idx[p], c = idx[q];
                        if (c > r) std::swap(r, c);
                        at(r, c) += cf[p] * cf[q];
                    }
            }
    }
    // the loop above adds the off-diagonal once per unordered (p, q); the
    // diagonal terms (p == q) once as well -- which is A^T A exactly.
    // A grid point with no antenna is not an unknown: its (empty) row gets a
    // unit diagonal, so it adds no null direction.
    for (int a = 0; a < N; ++a)
        if (!bit_of(bits, a)) at(a, a) = 1.0;
    std::vector<double> D(V, 0.0), diag0(V);
    for (int r = 0; r < V; ++r) diag0[r] = at(r, r);
    int null = 0;
    for (int r = 0; r < V; ++r) {
        const int fr = first[r];
        for (int c = fr; c < r; ++c) {
            const int lo = std::max(fr, first[c]);
            double s = at(r, c);
            for (int k = lo; k < c; ++k) s -= at(r, k) * D[k] * at(c, k);
            at(r, c) = (D[c] != 0.0) ? s / D[c] : 0.0;
        }
        double d = at(r, r);
        for (int k = fr; k < r; ++k) d -= at(r, k) * at(r, k) * D[k];
        if (d <= 1e-9 * std::max(1.0, diag0[r])) {
            ++null;
            d = 0.0;
        }
        D[r] = d;
        at(r, r) = 1.0;
    }
    return null;
}

int build_sel(int n, const int32_t* types_xy, int k, Sel& s, const uint32_t* bits = nullptr) {
    if (n < 2 || n > RRC_MAX_GRID || k < 1 || k > RRC_MAX_TYPES || !types_xy) return RRC_EINVAL;
    std::memset(&s, 0, sizeof(s));
    s.n = n;
    s.N = n * n;
    s.K = k;
    int off = 0;
    for (int t = 0; t < k; ++t) {
        const int dx = types_xy[2 * t], dy = types_xy[2 * t + 1];
        if (!valid_type(n, dx, dy)) return RRC_EINVAL;
        for (int u = 0; u < t; ++u)
            if (s.dx[u] == dx && s.dy[u] == dy) return RRC_EINVAL;
        s.dx[t] = dx;
        s.dy[t] = dy;
        s.off[t] = off;
        const long m = group_size_masked(n, bits, dx, dy);
        if (m == 0) return RRC_EINVAL;    // a type no pair realises
        off += (int)m;
    }
    s.off[k] = off;
    s.P = off;
    return RRC_OK;
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

}  // namespace

namespace rrc {

// Scratch of rrc_run_static: a file-scope device array, one copy per GPU,
// held until the process ends.  Host code never passes `scratch` itself to
// a kernel (in host code the name is only a host-side stand-in); it uses the
// device address hipGetSymbolAddress returns for the device current when it
// is looked up, kept per device in scratch_ptr.
static __device__ __align__(256) unsigned char scratch[RRC_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
static void* scratch_ptr[kMaxDevices] = {nullptr};
static std::mutex scratch_mu;

// The scratch address on `dev`, which must be the current device; looked up
// once per device.
static void* device_scratch(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
        scratch_ptr[dev] = ptr;
    }
    return scratch_ptr[dev];
}

// stamps[0] = now; stamps[1 .. U] = 0 (raised by each stage's atomic max)
__global__ __launch_bounds__(256) void k_stamp_start(unsigned long long* stamps, int n_units) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q == 0) stamps[0] = (unsigned long long)wall_clock64();
    else if (q <= n_units) stamps[q] = 0ull;
}

hipError_t launch_stamp_start(unsigned long long* stamps, int n_units, hipStream_t st) {
    hipLaunchKernelGGL(k_stamp_start, dim3((unsigned)((n_units + 256) / 256)), dim3(256), 0, st, stamps, n_units);
    return hipGetLastError();
}

// Copy of n8 8-byte words (complex64 arrays), one per work-item.
__global__ __launch_bounds__(256) void k_copy(uint2* __restrict__ dst, const uint2* __restrict__ src, size_t n8) {
    const size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n8) dst[q] = src[q];
}

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t st) {
    const size_t n8 = bytes / 8;
    if (n8 == 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)((n8 + 255) / 256)), dim3(256), 0, st, static_cast<uint2*>(dst),
                       static_cast<const uint2*>(src), n8);
    return hipGetLastError();
}

}  // namespace rrc

extern "C" {

void rrc_default_opts(rrc_solver_opts* o) {
    if (!o) return;
    o->init_mode = RRC_INIT_FIRSTCAL;
    o->degen_mode = RRC_DEGEN_REFANT;
    o->max_gn = 12;
    o->fp64_steps = 1;
    o->max_cg = 400;
    o->cg_tol = 1e-2f;
    o->tol32 = 1e-5f;
}

const char* rrc_strerror(int code) {
    switch (code) {
        case RRC_OK: return "ok";
        case RRC_EINVAL: return "invalid argument";
        case RRC_EDEGEN: return "selection has more than the four redundant-calibration degeneracies";
        case RRC_EDEVICE: return "HIP runtime error";
        case RRC_ENOTIMPL: return "not implemented";
        case RRC_ERANGE: return "size beyond a limit";
        default: return "unknown error";
    }
}

int rrc_degeneracy_count(int32_t n, const int32_t* types_xy, int32_t k, int32_t* n_null_amp,
                         int32_t* n_null_phase) {
    Sel s;
    const int rc = build_sel(n, types_xy, k, s);
    if (rc != RRC_OK) return rc;
    if (!n_null_amp || !n_null_phase) return RRC_EINVAL;
    std::vector<Type> sel(k);
    for (int t = 0; t < k; ++t) sel[t] = {s.dx[t], s.dy[t]};
    *n_null_amp = normal_nullity(n, sel, +1);
    *n_null_phase = normal_nullity(n, sel, -1);
    return RRC_OK;
}

int rrc_select_subset(int32_t n, double p, double log_base, int32_t* types_xy, int32_t cap,
                      int32_t* k_out, int32_t* n_pairs_out) {
    if (n < 2 || n > RRC_MAX_GRID || !(p > 0.0) || !types_xy || !k_out || !n_pairs_out)
        return RRC_EINVAL;
    const std::vector<Type> all = sorted_types(n);
    const double N = (double)n * n;
    const double lg = (log_base > 1.0) ? std::log(N) / std::log(log_base) : std::log(N);
    const double budget = p * N * lg;
    long cum = 0;
    int best = 1;
    double best_d = 1e300;
    for (size_t t = 0; t < all.size(); ++t) {
        cum += group_size(n, all[t].dx, all[t].dy);
        const double d = std::fabs((double)cum - budget);
        if (d < best_d) {
            best_d = d;
            best = (int)t + 1;
        }
    }
    int k = best;
    std::vector<int32_t> xy;
    while (true) {
        xy.clear();
        for (int t = 0; t < k; ++t) {
            xy.push_back(all[t].dx);
            xy.push_back(all[t].dy);
        }
        if (k > RRC_MAX_TYPES) return RRC_ERANGE;
        int32_t na = 0, np = 0;
        const int rc = rrc_degeneracy_count(n, xy.data(), k, &na, &np);
        if (rc != RRC_OK) return rc;
        if (na + np == 4) break;
        if (k >= (int)all.size()) return RRC_EDEGEN;
        ++k;
    }
    if (k > cap) return RRC_ERANGE;
    long pairs = 0;
    for (int t = 0; t < k; ++t) {
        types_xy[2 * t] = all[t].dx;
        types_xy[2 * t + 1] = all[t].dy;
        pairs += group_size(n, all[t].dx, all[t].dy);
    }
    *k_out = k;
    *n_pairs_out = (int32_t)pairs;
    return RRC_OK;
}

static int plan_create(rrc_plan** out, int32_t n, const int32_t* types_xy, int32_t k, int32_t n_units,
                       int32_t n_time, int32_t dtype, const rrc_solver_opts* opts, const uint8_t* mask) {
    if (!out) return RRC_EINVAL;
    *out = nullptr;
    uint32_t bits_store[rrc::kMaskWords];
    const uint32_t* bits = nullptr;
    int n_live = n * n, ref0 = 0;
    if (mask) {
        if (n < 2 || n > RRC_MAX_GRID) return RRC_EINVAL;
        pack_mask(n, mask, bits_store);
        bits = bits_store;
        n_live = 0;
        ref0 = -1;
        for (int a = 0; a < n * n; ++a)
            if (mask[a]) {
                ++n_live;
                if (ref0 < 0) ref0 = a;
            }
        // the references of the degeneracy fix: the first antenna and its
        // +x and +y neighbours
        if (ref0 < 0 || ref0 % n + 1 >= n || ref0 / n + 1 >= n || !mask[ref0 + 1] || !mask[ref0 + n])
            return RRC_EINVAL;
    }
    Sel s;
    int rc = build_sel(n, types_xy, k, s, bits);
    if (rc != RRC_OK) return rc;
    if (n_units < 1 || n_time < 1 || (dtype != RRC_C64 && dtype != RRC_CI4)) return RRC_EINVAL;
    if (dtype == RRC_CI4 && (long)n_time * 98L > 2147483647L) return RRC_ERANGE;
    rrc_solver_opts o;
    rrc_default_opts(&o);
    if (opts) o = *opts;
    if (o.max_gn < 1 || o.fp64_steps < 0 || o.max_cg < 1 || !(o.cg_tol > 0.f) ||
        (o.init_mode != RRC_INIT_FIRSTCAL && o.init_mode != RRC_INIT_GAINS) ||
        (o.degen_mode != RRC_DEGEN_REFANT && o.degen_mode != RRC_DEGEN_MATCH))
        return RRC_EINVAL;
    bool has10 = false, has01 = false;
    for (int t = 0; t < k; ++t) {
        has10 |= (s.dx[t] == 1 && s.dy[t] == 0);
        has01 |= (s.dx[t] == 0 && s.dy[t] == 1);
    }
    if (!mask && o.init_mode == RRC_INIT_FIRSTCAL && !(has10 && has01)) return RRC_EINVAL;
    {
        std::vector<Type> sv(k);
        for (int t = 0; t < k; ++t) sv[t] = {s.dx[t], s.dy[t]};
        if (normal_nullity(n, sv, +1, bits) + normal_nullity(n, sv, -1, bits) != 4) return RRC_EDEGEN;
    }

    rrc_plan* p = new (std::nothrow) rrc_plan();
    if (!p) return RRC_ERANGE;
    p->sel = s;
    if (mask) {
        p->masked = true;
        std::memcpy(p->mask_bits, bits_store, sizeof(bits_store));
    }
    p->n_live = n_live;
    p->ref0 = ref0;
    // FFT size: the smallest the kernels instantiate (16, 32, 48, 64, 96,
    // 128) with M >= 2n - 1, so the lags -(n-1) .. n-1 never wrap round;
    // the next power of two, where it differs, is the alternative a caller
    // or the tuner may choose.  The workspace holds either.
    int Mp = 16;
    while (Mp < 2 * n) Mp *= 2;
    int M = Mp;
    for (const int c : {48, 96})
        if (c >= 2 * n - 1 && c < M) M = c;
    p->M = M;
    p->M_default = M;
    p->M_alt = M != Mp ? Mp : 0;
    p->nlag = 2 * n * (n - 1);
    p->U = n_units;
    p->T = n_time;
    p->dtype = dtype;
    p->opts = o;

    // FFT-correlator: aim for >= 2048 workgroups, each doing >= 4 steps
    const int S = rrc::fft_samples_per_step_for(M);
    int nch = std::max(1, std::min(ceil_div(2048, n_units), n_time / (4 * S)));
    int tch = ceil_div(ceil_div(n_time, nch), S) * S;
    p->fft_tchunk = tch;
    p->fft_nchunk = ceil_div(n_time, tch);
    p->fft_tchunk0 = tch;

    // X-engine: blocks of 512 (4-bit) or 256 antennas, S samples staged per step, time
    // chunks (whole steps) so that the launch has >= 2048 workgroups while
    // each still runs >= 4 steps and >= 64 samples (fewer chunk partials
    // for the finishing pass to add)
    {
        int halo = 0;
        for (int t = 0; t < s.K; ++t) halo = std::max(halo, s.dy[t] * s.n + s.dx[t]);
        const int apb = rrc::xengine_antennas_per_block(dtype == RRC_CI4);
        // staging limits of the X-engine: partners within 248 antennas in
        // raster order, and whole 32-bit words of 4-bit samples
        if (halo > rrc::xengine_max_halo() || (dtype == RRC_CI4 && (s.N & 3))) {
            delete p;
            return RRC_ENOTIMPL;
        }
        p->x_halo = halo;
        p->x_nablk = ceil_div(s.N, apb);
        p->x_S = rrc::xengine_samples_per_step(dtype == RRC_CI4);
        const long wg = (long)n_units * p->x_nablk;
        const long want = wg >= 2048 ? 1 : ceil_div(2048, (int)wg);
        const int xn = (int)std::max(1L, std::min(want, (long)(n_time / std::max(4 * p->x_S, 64))));
        const int xt = ceil_div(ceil_div(n_time, xn), p->x_S) * p->x_S;
        p->x_tchunk = xt;
        p->x_nchunk = ceil_div(n_time, xt);
        if (dtype == RRC_CI4 && !mask) {
            p->x_mf.sel = s;
            p->x_mf_ok = rrc::xmfma_plan(s, p->x_mf) && xt % 32 == 0 && xt <= (1 << 17);
        }
    }

    // solver
    // the solver's state always fits in LDS (131 KB at 4096 antennas);
    // V^reduced joins it when there is room, on one-antenna-per-work-item
    // shapes (up to 512 antennas)
    p->solve_vcache = s.N <= 512 && rrc::solve_lds_bytes(s, true) <= 150 * 1024;
    p->solve_lds_bytes = rrc::solve_lds_bytes(s, p->solve_vcache);

    size_t off = 0;
    p->off_fft = off;
    off = align256(off + (size_t)n_units * p->fft_nchunk * Mp * Mp * sizeof(float));
    if (M == 96) {
        p->off_hinv = off;
        off = align256(off + (size_t)n_units * 48 * 48 * 8);
    }
    p->off_x = off;
    off = align256(off + (p->x_nchunk > 1 ? (size_t)n_units * p->x_nchunk * s.P * 8 : 0));
    p->off_gcopy = off;                      // copy of gains_in when it aliases gains_out
    off = align256(off + (size_t)n_units * s.N * 8);
    if (mask) {                              // the masked lattice's tables
        p->off_live = off;
        off = align256(off + (size_t)s.N);
        p->off_pidx = off;
        off = align256(off + (size_t)s.K * s.N * 4);
        p->off_pfirst = off;
        off = align256(off + (size_t)s.P * 4);
        p->off_nd = off;
        off = align256(off + (size_t)p->nlag * 4);
    }
    p->ws_bytes = off;
    *out = p;
    return RRC_OK;
}

int rrc_plan_create(rrc_plan** out, int32_t n, const int32_t* types_xy, int32_t k, int32_t n_units,
                    int32_t n_time, int32_t dtype, const rrc_solver_opts* opts) {
    return plan_create(out, n, types_xy, k, n_units, n_time, dtype, opts, nullptr);
}

int rrc_plan_create_masked(rrc_plan** out, int32_t n, const uint8_t* mask, const int32_t* types_xy, int32_t k,
                           int32_t n_units, int32_t n_time, int32_t dtype, const rrc_solver_opts* opts) {
    if (!mask) return RRC_EINVAL;
    return plan_create(out, n, types_xy, k, n_units, n_time, dtype, opts, mask);
}

int rrc_hex_mask(int32_t side, uint8_t* mask, int32_t cap, int32_t* n_out, int32_t* n_live_out) {
    if (side < 2 || !mask || !n_out || !n_live_out) return RRC_EINVAL;
    const int n = 2 * side - 1, r = side - 1;
    if (n > RRC_MAX_GRID) return RRC_ERANGE;
    if (cap < n * n) return RRC_ERANGE;
    int live = 0;
    for (int y = 0; y < n; ++y)
        for (int x = 0; x < n; ++x) {
            const int a = x - r, b = y - r;      // axial coordinates
            const bool on = std::abs(a + b) <= r;
            mask[y * n + x] = on ? 1 : 0;
            live += on;
        }
    *n_out = n;
    *n_live_out = live;
    return RRC_OK;
}

int rrc_degeneracy_count_masked(int32_t n, const uint8_t* mask, const int32_t* types_xy, int32_t k,
                                int32_t* n_null_amp, int32_t* n_null_phase) {
    if (!mask || !n_null_amp || !n_null_phase || n < 2 || n > RRC_MAX_GRID) return RRC_EINVAL;
    uint32_t bits[rrc::kMaskWords];
    pack_mask(n, mask, bits);
    Sel s;
    const int rc = build_sel(n, types_xy, k, s, bits);
    if (rc != RRC_OK) return rc;
    std::vector<Type> sel(k);
    for (int t = 0; t < k; ++t) sel[t] = {s.dx[t], s.dy[t]};
    *n_null_amp = normal_nullity(n, sel, +1, bits);
    *n_null_phase = normal_nullity(n, sel, -1, bits);
    return RRC_OK;
}

int rrc_select_subset_masked(int32_t n, const uint8_t* mask, int32_t metric, double p, double log_base,
                             int32_t* types_xy, int32_t cap, int32_t* k_out, int32_t* n_pairs_out) {
    if (n < 2 || n > RRC_MAX_GRID || !mask || !(p > 0.0) || !types_xy || !k_out || !n_pairs_out ||
        (metric != RRC_METRIC_SQUARE && metric != RRC_METRIC_HEX))
        return RRC_EINVAL;
    uint32_t bits[rrc::kMaskWords];
    pack_mask(n, mask, bits);
    int live = 0;
    for (int a = 0; a < n * n; ++a) live += mask[a] != 0;
    if (live < 2) return RRC_EINVAL;
    // types some pair realises, in ascending length under the metric
    std::vector<Type> all;
    std::vector<long> size;
    for (const Type& t : sorted_types(n, metric)) {
        const long m = group_size_masked(n, bits, t.dx, t.dy);
        if (m > 0) {
            all.push_back(t);
            size.push_back(m);
        }
    }
    const double N = (double)live;
    const double lg = (log_base > 1.0) ? std::log(N) / std::log(log_base) : std::log(N);
    const double budget = p * N * lg;
    long cum = 0;
    int best = 1;
    double best_d = 1e300;
    for (size_t t = 0; t < all.size(); ++t) {
        cum += size[t];
        const double d = std::fabs((double)cum - budget);
        if (d < best_d) {
            best_d = d;
            best = (int)t + 1;
        }
    }
    int k = best;
    while (true) {
        if (k > RRC_MAX_TYPES) return RRC_ERANGE;
        std::vector<Type> sel(all.begin(), all.begin() + k);
        if (normal_nullity(n, sel, +1, bits) + normal_nullity(n, sel, -1, bits) == 4) break;
        if (k >= (int)all.size()) return RRC_EDEGEN;
        ++k;
    }
    if (k > cap) return RRC_ERANGE;
    long pairs = 0;
    for (int t = 0; t < k; ++t) {
        types_xy[2 * t] = all[t].dx;
        types_xy[2 * t + 1] = all[t].dy;
        pairs += size[t];
    }
    *k_out = k;
    *n_pairs_out = (int32_t)pairs;
    return RRC_OK;
}

static void release_device(rrc_plan* p) {
    if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
    if (p->ev_join) (void)hipEventDestroy(p->ev_join);
    if (p->aux) (void)hipStreamDestroy(p->aux);
    p->aux = nullptr;
    p->ev_fork = p->ev_join = nullptr;
    p->scratch = nullptr;
    p->prepared = false;
    p->device = -1;
}

static rrc::SolveLaunch solve_launch(const rrc_plan* p);

// Device resources of a plan, made once on the device current at the first
// device call, so that later calls enqueue launches and event operations
// only (and can be captured into a graph by the caller).
static int prepare(rrc_plan* p) {
    if (p->prepared) return RRC_OK;
    int dev = -1, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return RRC_EDEVICE;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return RRC_EDEVICE;
    if (hipStreamCreateWithFlags(&p->aux, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_join, hipEventDisableTiming) != hipSuccess ||
        rrc::prepare_solve(solve_launch(p)) != hipSuccess) {
        release_device(p);
        return RRC_EDEVICE;
    }
    p->cu_count = cus;
    p->device = dev;
    // the static scratch's address on this device (rrc_run_static); null
    // if the lookup fails, which only that entry point reports
    p->scratch = rrc::device_scratch(dev);
    p->prepared = true;
    return RRC_OK;
}

void rrc_plan_destroy(rrc_plan* p) {
    if (!p) return;
    release_device(p);
    delete p;
}

int rrc_plan_set_order(rrc_plan* p, int32_t order) {
    if (!p || order < RRC_ORDER_XENG_FIRST || order > RRC_ORDER_SERIAL) return RRC_EINVAL;
    p->order = order;
    return RRC_OK;
}

// FFT sizes of a plan: the default, or the power of two beside it.  The
// default's samples per step are a multiple of the alternative's, so its
// time chunks suit both, and the workspace holds the larger grid.
static bool fft_size_ok(const rrc_plan* p, int M) {
    return M == p->M_default || (p->M_alt != 0 && M == p->M_alt);
}

int rrc_plan_set_fft_size(rrc_plan* p, int32_t M) {
    if (!p || !fft_size_ok(p, M)) return RRC_EINVAL;
    p->M = M;
    return RRC_OK;
}

int rrc_plan_set_xengine(rrc_plan* p, int32_t kind) {
    if (!p || (kind != RRC_XENG_AUTO && kind != RRC_XENG_DOT && kind != RRC_XENG_MFMA)) return RRC_EINVAL;
    if (kind == RRC_XENG_MFMA && !p->x_mf_ok) return RRC_ENOTIMPL;
    p->x_kind = kind;
    return RRC_OK;
}

int rrc_plan_prepare(rrc_plan* p) {
    if (!p) return RRC_EINVAL;
    return prepare(p);
}

int rrc_plan_get_info(const rrc_plan* p, rrc_plan_info* info) {
    if (!p || !info) return RRC_EINVAL;
    info->n = p->sel.n;
    info->n_ant = p->sel.N;
    info->fft_size = p->M;
    info->n_lags = p->nlag;
    info->n_types = p->sel.K;
    info->n_pairs = p->sel.P;
    info->dof = p->sel.P - p->sel.N - p->sel.K + 2;
    info->n_units = p->U;
    info->n_time = p->T;
    info->dtype = p->dtype;
    info->workspace_bytes = p->ws_bytes;
    info->n_live = p->n_live;
    info->masked = p->masked ? 1 : 0;
    if (p->masked) info->dof = p->sel.P - p->n_live - p->sel.K + 2;
    return RRC_OK;
}

int rrc_workspace_size(const rrc_plan* p, size_t* bytes) {
    if (!p || !bytes) return RRC_EINVAL;
    *bytes = p->ws_bytes;
    return RRC_OK;
}

// A masked plan's tables, rebuilt in the workspace from the mask bits;
// returns the pointers the kernels read (all null for a full grid).
static int mask_tables(const rrc_plan* p, void* stream, void* d_work, rrc::MaskTables& mt, bool build = true) {
    mt = rrc::MaskTables{};
    mt.n_live = p->n_live;
    mt.ref0 = p->ref0;
    if (!p->masked) return RRC_OK;
    char* w = static_cast<char*>(d_work);
    rrc::MaskLaunch L;
    L.sel = p->sel;
    std::memcpy(L.bits, p->mask_bits, sizeof(L.bits));
    L.live = reinterpret_cast<uint8_t*>(w + p->off_live);
    L.pidx = reinterpret_cast<int*>(w + p->off_pidx);
    L.pfirst = reinterpret_cast<int*>(w + p->off_pfirst);
    L.nd = reinterpret_cast<float*>(w + p->off_nd);
    if (build && rrc::launch_mask_tables(L, as_stream(stream)) != hipSuccess) return RRC_EDEVICE;
    mt.live = L.live;
    mt.pidx = L.pidx;
    mt.pfirst = L.pfirst;
    mt.nd = L.nd;
    return RRC_OK;
}

static int fftcorr_impl(rrc_plan* p, void* stream, const void* d_volt, const void* d_gains,
                        void* d_vunique, float* d_vauto, void* d_work, uint64_t* d_stamps, bool build = true) {
    if (!p || !d_volt || !d_gains || !d_vunique || !d_vauto || !d_work) return RRC_EINVAL;
    rrc::FftLaunch L{};
    L.stamps = reinterpret_cast<unsigned long long*>(d_stamps);
    L.M = p->M;
    L.n = p->sel.n;
    L.T = p->T;
    L.n_units = p->U;
    L.tchunk = p->fft_tchunk;
    L.nchunk = p->fft_nchunk;
    L.ci4 = p->dtype == RRC_CI4;
    L.volt = d_volt;
    L.gains = reinterpret_cast<const float2*>(d_gains);
    L.ppart = reinterpret_cast<float*>(static_cast<char*>(d_work) + p->off_fft);
    L.hinv = p->off_hinv ? reinterpret_cast<float2*>(static_cast<char*>(d_work) + p->off_hinv) : nullptr;
    L.vunique = reinterpret_cast<float2*>(d_vunique);
    L.vauto = d_vauto;
    const int rc = mask_tables(p, stream, d_work, L.mt, build);
    if (rc != RRC_OK) return rc;
    return rrc::launch_fftcorr(L, as_stream(stream)) == hipSuccess ? RRC_OK : RRC_EDEVICE;
}

int rrc_fftcorr(rrc_plan* p, void* stream, const void* d_volt, const void* d_gains, void* d_vunique,
                float* d_vauto, void* d_work) {
    return fftcorr_impl(p, stream, d_volt, d_gains, d_vunique, d_vauto, d_work, nullptr);
}

static int xengine_impl(rrc_plan* p, void* stream, const void* d_volt, void* d_vred, void* d_work, bool build) {
    if (!p || !d_volt || !d_vred || !d_work) return RRC_EINVAL;
    rrc::XengLaunch L;
    L.sel = p->sel;
    L.T = p->T;
    L.n_units = p->U;
    L.tchunk = p->x_tchunk;
    L.nchunk = p->x_nchunk;
    L.nablk = p->x_nablk;
    L.halo = p->x_halo;
    L.inv_t = 1.0f / (float)p->T;
    L.ci4 = p->dtype == RRC_CI4;
    L.volt = d_volt;
    L.vpart = static_cast<char*>(d_work) + p->off_x;
    L.vred = d_vred;
    // the matrix-core form only on request: at the 64x64 grid's banded
    // selection it takes 27.7 ms per 1024 units against 10.7 ms for the
    // dot-product kernel (LDS-bound, one workgroup per CU)
    L.mfma = L.ci4 && p->x_mf_ok && p->x_kind == RRC_XENG_MFMA;
    if (L.mfma) {
        L.mf_inst = p->x_mf.mf_inst;
        L.mf_nrun = p->x_mf.mf_nrun;
        for (int r = 0; r < rrc::kXMaxRuns; ++r) {
            L.mf_start[r] = p->x_mf.mf_start[r];
            L.mf_len[r] = p->x_mf.mf_len[r];
        }
        L.mf_lo = p->x_mf.mf_lo;
        L.mf_cnt = p->x_mf.mf_cnt;
    }
    const int rc = mask_tables(p, stream, d_work, L.mt, build);
    if (rc != RRC_OK) return rc;
    return rrc::launch_xengine(L, as_stream(stream)) == hipSuccess ? RRC_OK : RRC_EDEVICE;
}

int rrc_xengine(rrc_plan* p, void* stream, const void* d_volt, void* d_vred, void* d_work) {
    return xengine_impl(p, stream, d_volt, d_vred, d_work, true);
}

static rrc::SolveLaunch solve_launch(const rrc_plan* p) {
    rrc::SolveLaunch L{};
    L.sel = p->sel;
    L.n_units = p->U;
    L.ci4 = p->dtype == RRC_CI4;
    L.vcache = p->solve_vcache;
    L.lds_bytes = p->solve_lds_bytes;
    L.o = {p->opts.init_mode, p->opts.degen_mode, p->opts.max_gn, p->opts.fp64_steps,
           p->opts.max_cg, p->opts.cg_tol, p->opts.tol32};
    return L;
}

static int solve_impl(rrc_plan* p, void* stream, const void* d_vred, const void* d_gains_in,
                      const void* d_gains_ref, void* d_gains_out, void* d_vmodel, float* d_chisq,
                      int32_t* d_niter, int32_t* d_status, uint64_t* d_stamps, void* d_work, bool build) {
    if (!p || !d_vred || !d_gains_out || !d_vmodel || !d_chisq || !d_niter || !d_status)
        return RRC_EINVAL;
    // a masked lattice starts from the caller's gains (FIRSTCAL chains
    // phases along full grid rows and columns) and needs the workspace for
    // its pair tables
    if (p->masked && p->opts.init_mode != RRC_INIT_GAINS) return RRC_ENOTIMPL;
    if (p->masked && !d_work) return RRC_EINVAL;
    if (p->opts.init_mode == RRC_INIT_GAINS && !d_gains_in) return RRC_EINVAL;
    if (p->opts.degen_mode == RRC_DEGEN_MATCH && !d_gains_ref) return RRC_EINVAL;
    const int rc = prepare(p);
    if (rc != RRC_OK) return rc;
    rrc::SolveLaunch L = solve_launch(p);
    L.exclusive = (p->concurrent_units > 0 ? p->concurrent_units : p->U) <= p->cu_count;
    L.vred = d_vred;
    L.gains_in = reinterpret_cast<const float2*>(d_gains_in);
    L.gains_ref = reinterpret_cast<const float2*>(d_gains_ref);
    L.gains_out = reinterpret_cast<float2*>(d_gains_out);
    L.vmodel = reinterpret_cast<float2*>(d_vmodel);
    L.chisq = d_chisq;
    L.niter = d_niter;
    L.status = d_status;
    L.stamps = reinterpret_cast<unsigned long long*>(d_stamps);
    const int rm = mask_tables(p, stream, d_work, L.mt, build);
    if (rm != RRC_OK) return rm;
    return rrc::launch_solve(L, as_stream(stream)) == hipSuccess ? RRC_OK : RRC_EDEVICE;
}

int rrc_solve(rrc_plan* p, void* stream, const void* d_vred, const void* d_gains_in,
              const void* d_gains_ref, void* d_gains_out, void* d_vmodel, float* d_chisq,
              int32_t* d_niter, int32_t* d_status, void* d_work) {
    // the solve keeps its whole state in LDS; d_work holds a masked
    // lattice's pair tables
    return solve_impl(p, stream, d_vred, d_gains_in, d_gains_ref, d_gains_out, d_vmodel, d_chisq,
                      d_niter, d_status, nullptr, d_work, true);
}

int rrc_omnical(rrc_plan* p, void* stream, const void* d_vred, const void* d_gains_in, int32_t max_iter,
                float tol, int32_t finish, void* d_gains, void* d_vmodel, float* d_chisq, int32_t* d_niter,
                int32_t* d_status, float* d_delta, void* d_work) {
    if (!p || !d_vred || !d_gains || !d_vmodel || !d_niter || !d_status || max_iter < 0 || !(tol >= 0.f))
        return RRC_EINVAL;
    if (finish && !d_chisq) return RRC_EINVAL;
    if (p->masked && !d_work) return RRC_EINVAL;
    rrc::OmniLaunch L{};
    L.n = p->sel.n;
    L.K = p->sel.K;
    L.P = p->sel.P;
    L.n_units = p->U;
    L.all = false;
    L.ci4 = p->dtype == RRC_CI4;
    L.sel = p->sel;
    L.lds_types = 0;
    L.max_iter = max_iter;
    L.tol = tol;
    L.damping = 0.3f;
    L.finish = finish != 0;
    L.gains_in = reinterpret_cast<const float2*>(d_gains_in);
    L.vred = d_vred;
    L.gains = d_gains;
    L.vmodel = d_vmodel;
    L.chisq = d_chisq;
    L.niter = d_niter;
    L.status = d_status;
    L.delta = d_delta;
    const int rc = mask_tables(p, stream, d_work, L.mt);
    if (rc != RRC_OK) return rc;
    return rrc::launch_omnical(L, as_stream(stream)) == hipSuccess ? RRC_OK : RRC_EDEVICE;
}

static int chisq_common(rrc_plan* p, void* stream, const void* d_g, const void* d_vm,
                        const void* d_vred, float* d_chisq, void* d_grad_g, void* d_grad_v,
                        float* d_diag_g, float* d_diag_v, bool adj) {
    if (!p || !d_g || !d_vm || !d_vred) return RRC_EINVAL;
    if (!adj && !d_chisq) return RRC_EINVAL;
    if (p->masked) return RRC_ENOTIMPL;
    rrc::ChisqLaunch L;
    L.sel = p->sel;
    L.n_units = p->U;
    L.g = reinterpret_cast<const float2*>(d_g);
    L.vm = reinterpret_cast<const float2*>(d_vm);
    L.vred = reinterpret_cast<const float2*>(d_vred);
    L.chisq = d_chisq;
    L.grad_g = reinterpret_cast<float2*>(d_grad_g);
    L.grad_v = reinterpret_cast<float2*>(d_grad_v);
    L.diag_g = d_diag_g;
    L.diag_v = d_diag_v;
    return rrc::launch_chisq(L, as_stream(stream), adj) == hipSuccess ? RRC_OK : RRC_EDEVICE;
}

int rrc_chisq_fwd(rrc_plan* p, void* stream, const void* d_g, const void* d_vm, const void* d_vred,
                  float* d_chisq) {
    return chisq_common(p, stream, d_g, d_vm, d_vred, d_chisq, nullptr, nullptr, nullptr, nullptr,
                        false);
}

int rrc_chisq_adj(rrc_plan* p, void* stream, const void* d_g, const void* d_vm, const void* d_vred,
                  void* d_grad_g, void* d_grad_v, float* d_diag_g, float* d_diag_v) {
    return chisq_common(p, stream, d_g, d_vm, d_vred, nullptr, d_grad_g, d_grad_v, d_diag_g,
                        d_diag_v, true);
}

int rrc_run(rrc_plan* p, void* stream, int32_t mode, const rrc_io* io) {
    if (!p || !io) return RRC_EINVAL;
    if (p->masked && p->opts.init_mode != RRC_INIT_GAINS) return RRC_ENOTIMPL;
    if (mode != RRC_RUN_PIPELINED && mode != RRC_RUN_SELFCAL) return RRC_EINVAL;
    if (mode == RRC_RUN_PIPELINED && !io->d_gains_in) return RRC_EINVAL;
    if (!io->d_volt || !io->d_vunique || !io->d_vauto || !io->d_vred || !io->d_gains_out ||
        !io->d_vmodel || !io->d_chisq || !io->d_niter || !io->d_status || !io->d_work)
        return RRC_EINVAL;
    if (p->opts.init_mode == RRC_INIT_GAINS && !io->d_gains_in) return RRC_EINVAL;
    if (p->opts.degen_mode == RRC_DEGEN_MATCH && !io->d_gains_ref) return RRC_EINVAL;
    int rc = prepare(p);
    if (rc != RRC_OK) return rc;
    hipStream_t st = as_stream(stream);
    char* work = static_cast<char*>(io->d_work);
    if (io->d_stamps && rrc::launch_stamp_start(reinterpret_cast<unsigned long long*>(io->d_stamps),
                                                p->U, st) != hipSuccess)
        return RRC_EDEVICE;
    // a masked lattice's tables, built once on `stream` before anything
    // forks; the stages below only read them
    {
        rrc::MaskTables mt;
        rc = mask_tables(p, stream, io->d_work, mt, true);
        if (rc != RRC_OK) return rc;
    }
    if (mode == RRC_RUN_SELFCAL) {
        // X-engine, solve, then the FFT-correlator with the solved gains
        rc = xengine_impl(p, stream, io->d_volt, io->d_vred, io->d_work, false);
        if (rc == RRC_OK)
            rc = solve_impl(p, stream, io->d_vred, io->d_gains_in, io->d_gains_ref, io->d_gains_out,
                            io->d_vmodel, io->d_chisq, io->d_niter, io->d_status, io->d_stamps, io->d_work,
                            false);
        if (rc == RRC_OK)
            rc = fftcorr_impl(p, stream, io->d_volt, io->d_gains_out, io->d_vunique, io->d_vauto,
                              io->d_work, io->d_stamps, false);
        return rc;
    }
    // PIPELINED.  The FFT-correlator applies the previous integration's gains
    // on the plan's auxiliary stream, beside the X-engine and the solve on
    // `stream`.  When gains_in and gains_out overlap (the real-time loop
    // feeding the solution back), the solve would rewrite the gains while
    // FFT workgroups still read them, so the FFT reads a copy taken first.
    const void* gfft = io->d_gains_in;
    {
        const size_t gb = (size_t)p->U * p->sel.N * 8;
        const char* gi = static_cast<const char*>(io->d_gains_in);
        const char* go = static_cast<const char*>(io->d_gains_out);
        if (gi < go + gb && go < gi + gb) {
            void* copy = work + p->off_gcopy;
            if (rrc::launch_copy(copy, io->d_gains_in, gb, st) != hipSuccess) return RRC_EDEVICE;
            gfft = copy;
        }
    }
    if (p->order == RRC_ORDER_SERIAL) {
        // the three stages one after another on `stream`
        rc = xengine_impl(p, stream, io->d_volt, io->d_vred, io->d_work, false);
        if (rc == RRC_OK)
            rc = fftcorr_impl(p, stream, io->d_volt, gfft, io->d_vunique, io->d_vauto, io->d_work, io->d_stamps,
                              false);
        if (rc == RRC_OK)
            rc = solve_impl(p, stream, io->d_vred, io->d_gains_in, io->d_gains_ref, io->d_gains_out,
                            io->d_vmodel, io->d_chisq, io->d_niter, io->d_status, io->d_stamps, io->d_work,
                            false);
        return rc;
    }
    auto fork_fft = [&]() -> int {
        if (hipEventRecord(p->ev_fork, st) != hipSuccess) return RRC_EDEVICE;
        if (hipStreamWaitEvent(p->aux, p->ev_fork, 0) != hipSuccess) return RRC_EDEVICE;
        const int r = fftcorr_impl(p, p->aux, io->d_volt, gfft, io->d_vunique, io->d_vauto, io->d_work,
                                   io->d_stamps, false);
        if (r != RRC_OK) return r;
        return hipEventRecord(p->ev_join, p->aux) == hipSuccess ? RRC_OK : RRC_EDEVICE;
    };
    if (p->order == RRC_ORDER_FFT_FIRST) {
        // a VALU-bound FFT stage that dominates the step starts at once; the
        // X-engine and the solve follow on `stream` beside it
        rc = fork_fft();
        if (rc == RRC_OK) rc = xengine_impl(p, stream, io->d_volt, io->d_vred, io->d_work, false);
        if (rc == RRC_OK)
            rc = solve_impl(p, stream, io->d_vred, io->d_gains_in, io->d_gains_ref, io->d_gains_out,
                            io->d_vmodel, io->d_chisq, io->d_niter, io->d_status, io->d_stamps, io->d_work,
                            false);
    } else {
        // The X-engine heads the critical path; once it is done the FFT
        // runs beside the latency-bound solve.  The solve is queued first:
        // it follows the X-engine on its own stream and so takes its CUs
        // before the FFT's workgroups fill the device.
        rc = xengine_impl(p, stream, io->d_volt, io->d_vred, io->d_work, false);
        if (rc != RRC_OK) return rc;
        if (hipEventRecord(p->ev_fork, st) != hipSuccess) return RRC_EDEVICE;
        rc = solve_impl(p, stream, io->d_vred, io->d_gains_in, io->d_gains_ref, io->d_gains_out,
                        io->d_vmodel, io->d_chisq, io->d_niter, io->d_status, io->d_stamps, io->d_work, false);
        if (rc != RRC_OK) return rc;
        if (hipStreamWaitEvent(p->aux, p->ev_fork, 0) != hipSuccess) return RRC_EDEVICE;
        rc = fftcorr_impl(p, p->aux, io->d_volt, gfft, io->d_vunique, io->d_vauto, io->d_work,
                          io->d_stamps, false);
        if (rc == RRC_OK && hipEventRecord(p->ev_join, p->aux) != hipSuccess) rc = RRC_EDEVICE;
    }
    if (rc != RRC_OK) return rc;
    return hipStreamWaitEvent(st, p->ev_join, 0) == hipSuccess ? RRC_OK : RRC_EDEVICE;
}

int rrc_run_static(rrc_plan* p, void* stream, int32_t mode, const rrc_io* io) {
    if (!p || !io) return RRC_EINVAL;
    if (p->masked) return RRC_ENOTIMPL;
    if (io->d_work) return RRC_EINVAL;            // the scratch replaces the workspace
    if (p->ws_bytes > (size_t)RRC_STATIC_SCRATCH_BYTES) return RRC_ERANGE;
    // set-up (streams, events, the scratch address) belongs to
    // rrc_plan_prepare, so this call itself creates nothing
    if (!p->prepared) return RRC_EINVAL;
    if (!p->scratch) return RRC_EDEVICE;
    rrc_io io2 = *io;
    io2.d_work = p->scratch;
    return rrc_run(p, stream, mode, &io2);
}

// ------------------------------------------------------------------ tuner

// Chunk of `f` times the default chunk length, whole samples-per-step
// multiples: fewer partial grids, so the workspace still holds them.
static void set_fft_chunk_factor(rrc_plan* p, int f) {
    const int S = rrc::fft_samples_per_step_for(p->M);
    const int tch = std::min(ceil_div(p->T, S) * S, p->fft_tchunk0 * f);
    p->fft_tchunk = tch;
    p->fft_nchunk = ceil_div(p->T, tch);
}

static std::string tune_key(const rrc_plan* p) {
    hipDeviceProp_t prop{};
    std::string dev = "unknown";
    if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) dev = std::string(prop.gcnArchName) + "/" +
                                                                        std::to_string(prop.multiProcessorCount);
    std::string key = dev + " n=" + std::to_string(p->sel.n) + " types=";
    for (int t = 0; t < p->sel.K; ++t)
        key += std::to_string(p->sel.dx[t]) + ":" + std::to_string(p->sel.dy[t]) + (t + 1 < p->sel.K ? "," : "");
    key += " U=" + std::to_string(p->U) + " T=" + std::to_string(p->T) + " dtype=" + std::to_string(p->dtype);
    if (p->masked) {   // FNV-1a of the mask bits
        uint64_t h = 1469598103934665603ull;
        for (int w = 0; w < rrc::kMaskWords; ++w) {
            h ^= p->mask_bits[w];
            h *= 1099511628211ull;
        }
        char buf[32];
        std::snprintf(buf, sizeof(buf), " mask=%016llx", (unsigned long long)h);
        key += buf;
    }
    return key;
}

int rrc_plan_tune(rrc_plan* p, void* stream, const rrc_io* io, const char* cache_path, rrc_tune* out) {
    if (!p || !io || !out || !io->d_gains_in) return RRC_EINVAL;
    if (p->masked && p->opts.init_mode != RRC_INIT_GAINS) return RRC_ENOTIMPL;   // as rrc_run
    int rc = prepare(p);
    if (rc != RRC_OK) return rc;
    const std::string key = tune_key(p);
    // cached choice
    if (cache_path) {
        std::ifstream f(cache_path);
        std::string line;
        while (std::getline(f, line)) {
            const size_t bar = line.find(" | ");
            if (bar == std::string::npos || line.substr(0, bar) != key) continue;
            int fa = 0, ord = 0, xk = 0, mf = 0;
            float ms = 0.f;
            if (std::sscanf(line.c_str() + bar + 3, "chunk_factor=%d order=%d xengine=%d fft_size=%d ms=%f", &fa, &ord,
                            &xk, &mf, &ms) == 5 && fa >= 1 && fft_size_ok(p, mf)) {
                p->M = mf;
                set_fft_chunk_factor(p, fa);
                p->order = ord;
                p->x_kind = xk;
                *out = rrc_tune{fa, ord, xk, ms, 1, mf};
                return RRC_OK;
            }
        }
    }
    hipStream_t st = as_stream(stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return RRC_EDEVICE;
    }
    const int xkinds[2] = {RRC_XENG_DOT, RRC_XENG_MFMA};
    const int nx = (p->dtype == RRC_CI4 && p->x_mf_ok) ? 2 : 1;
    const int msizes[2] = {p->M_default, p->M_alt};
    const int nm = p->M_alt ? 2 : 1;
    rrc_tune best{1, RRC_ORDER_XENG_FIRST, RRC_XENG_AUTO, 1e30f, 0, p->M_default};
    for (int mi = 0; mi < nm && rc == RRC_OK; ++mi)
    for (int fa = 1; fa <= 4 && rc == RRC_OK; fa *= 2) {
        if (fa > 1 && p->fft_tchunk0 * (fa / 2) >= p->T) break;       // no fewer chunks left
        for (int ord = RRC_ORDER_XENG_FIRST; ord <= RRC_ORDER_SERIAL && rc == RRC_OK; ++ord)
            for (int xi = 0; xi < nx && rc == RRC_OK; ++xi) {
                p->M = msizes[mi];
                set_fft_chunk_factor(p, fa);
                p->order = ord;
                p->x_kind = nx > 1 ? xkinds[xi] : RRC_XENG_AUTO;
                rc = rrc_run(p, stream, RRC_RUN_PIPELINED, io);           // warm-up
                for (int r = 0; r < 3 && rc == RRC_OK; ++r) rc = rrc_run(p, stream, RRC_RUN_PIPELINED, io);
                if (rc != RRC_OK) break;
                if (hipEventRecord(e0, st) != hipSuccess) rc = RRC_EDEVICE;
                for (int r = 0; r < 3 && rc == RRC_OK; ++r) rc = rrc_run(p, stream, RRC_RUN_PIPELINED, io);
                float ms = 0.f;
                if (rc == RRC_OK && (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                                     hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
                    rc = RRC_EDEVICE;
                ms /= 3.f;
                if (rc == RRC_OK && ms < best.ms_per_run) best = rrc_tune{fa, ord, p->x_kind, ms, 0, p->M};
            }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    p->M = best.fft_size;
    set_fft_chunk_factor(p, best.fft_chunk_factor);
    p->order = best.order;
    p->x_kind = best.xengine;
    if (rc != RRC_OK) return rc;
    *out = best;
    if (cache_path) {
        std::ofstream f(cache_path, std::ios::app);
        char buf[160];
        std::snprintf(buf, sizeof(buf), " | chunk_factor=%d order=%d xengine=%d fft_size=%d ms=%.4f",
                      best.fft_chunk_factor, best.order, best.xengine, best.fft_size, best.ms_per_run);
        f << key << buf << "\n";
    }
    return RRC_OK;
}

// ------------------------------------------------------------------ batches

static void batch_release(rrc_batch* b) {
    for (hipEvent_t e : b->ev_done)
        if (e) (void)hipEventDestroy(e);
    for (hipStream_t s : b->branch)
        if (s) (void)hipStreamDestroy(s);
    if (b->ev_start) (void)hipEventDestroy(b->ev_start);
    b->ev_done.clear();
    b->branch.clear();
    b->ev_start = nullptr;
    b->prepared = false;
}

int rrc_batch_create(rrc_batch** out, int32_t n_plans, rrc_plan* const* plans, uint32_t flags) {
    if (!out) return RRC_EINVAL;
    *out = nullptr;
    if (n_plans < 1 || !plans || (flags & ~(uint32_t)RRC_BATCH_GRAPH)) return RRC_EINVAL;
    // Replaying the batch as a captured graph is switched off: capturing its
    // fork/join over the branch and auxiliary streams ended the process with
    // a host-side segmentation fault inside the runtime, and no cause in
    // this library has been shown.
    if (flags & RRC_BATCH_GRAPH) return RRC_ENOTIMPL;
    for (int i = 0; i < n_plans; ++i) {
        if (!plans[i]) return RRC_EINVAL;
        if (plans[i]->masked) return RRC_ENOTIMPL;   // batches run rrc_run
        for (int j = 0; j < i; ++j)
            if (plans[j] == plans[i]) return RRC_EINVAL;   // each plan owns its streams and events
    }
    rrc_batch* b = new (std::nothrow) rrc_batch();
    if (!b) return RRC_ERANGE;
    b->plans.assign(plans, plans + n_plans);
    b->flags = flags;
    *out = b;
    return RRC_OK;
}

void rrc_batch_destroy(rrc_batch* b) {
    if (!b) return;
    batch_release(b);
    delete b;
}

// Streams and events of a batch and of its plans, made on the first run.
static int batch_prepare(rrc_batch* b) {
    if (b->prepared) return RRC_OK;
    const int np = (int)b->plans.size();
    for (rrc_plan* p : b->plans) {
        const int rc = prepare(p);
        if (rc != RRC_OK) return rc;
    }
    b->branch.assign(np, nullptr);
    b->ev_done.assign(np, nullptr);
    bool ok = hipEventCreateWithFlags(&b->ev_start, hipEventDisableTiming) == hipSuccess;
    for (int i = 0; ok && i < np; ++i)
        ok = hipStreamCreateWithFlags(&b->branch[i], hipStreamNonBlocking) == hipSuccess &&
             hipEventCreateWithFlags(&b->ev_done[i], hipEventDisableTiming) == hipSuccess;
    if (!ok) {
        batch_release(b);
        return RRC_EDEVICE;
    }
    b->prepared = true;
    return RRC_OK;
}

// Fork every plan's run from `st` onto its branch stream and join them back.
static int batch_issue(rrc_batch* b, hipStream_t st, int32_t mode, const rrc_io* io) {
    const int np = (int)b->plans.size();
    long total = 0;
    for (rrc_plan* p : b->plans) total += p->U;
    if (hipEventRecord(b->ev_start, st) != hipSuccess) return RRC_EDEVICE;
    for (int i = 0; i < np; ++i) {
        rrc_plan* p = b->plans[i];
        if (hipStreamWaitEvent(b->branch[i], b->ev_start, 0) != hipSuccess) return RRC_EDEVICE;
        const long saved = p->concurrent_units;
        p->concurrent_units = total;
        const int rc = rrc_run(p, b->branch[i], mode, &io[i]);
        p->concurrent_units = saved;
        if (rc != RRC_OK) return rc;
        if (hipEventRecord(b->ev_done[i], b->branch[i]) != hipSuccess ||
            hipStreamWaitEvent(st, b->ev_done[i], 0) != hipSuccess)
            return RRC_EDEVICE;
    }
    return RRC_OK;
}

int rrc_batch_run(rrc_batch* b, void* stream, int32_t mode, const rrc_io* io) {
    if (!b || !io) return RRC_EINVAL;
    if (mode != RRC_RUN_PIPELINED && mode != RRC_RUN_SELFCAL) return RRC_EINVAL;
    const int rc = batch_prepare(b);
    if (rc != RRC_OK) return rc;
    return batch_issue(b, as_stream(stream), mode, io);
}

int rrc_wall_clock_hz(double* hz) {
    if (!hz) return RRC_EINVAL;
    int dev = -1, khz = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess || khz <= 0)
        return RRC_EDEVICE;
    *hz = 1e3 * (double)khz;
    return RRC_OK;
}

}  // extern "C"
