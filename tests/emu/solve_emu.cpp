// CPU build of the solver kernel's workgroup body (each work-item a
// fiber), exposed with a C interface for the host-side test-suite.
#define RRC_HOST_EMU
#include "../../paper_2005_03060_amd/csrc/solve.hip"

#include <vector>

using namespace rrc;

template <int NT, int APT, int KMAX>
static bool run_unit(const SolveLaunch& L, unsigned char* ldsbuf, int unit) {
    Shared<NT / 64> sh;
    return rrc_emu::run_group(NT, [&] { solve_unit<NT, APT, KMAX>(L, sh, ldsbuf, unit); });
}

template <int NT, int APT>
static bool run_shape(const SolveLaunch& L, unsigned char* ldsbuf, int unit) {
    if (L.sel.K <= 6) return run_unit<NT, APT, 6>(L, ldsbuf, unit);
    if (L.sel.K <= 8) return run_unit<NT, APT, 8>(L, ldsbuf, unit);
    if (L.sel.K <= 10) return run_unit<NT, APT, 10>(L, ldsbuf, unit);
    return run_unit<NT, APT, kMaxTypes>(L, ldsbuf, unit);
}

extern "C" int rrc_emu_solve(int n, const int* types_xy, int K, int U, int ci4, const void* vred,
                             const void* gains_in, const void* gains_ref, const int* iopts,
                             const float* fopts, void* gains_out, void* vmodel, float* chisq,
                             int* niter, int* status, int threads, int order, int vcache) {
    rrc_emu::group().order = order;
    rrc_emu::group().seed = 12345u;
    Sel s{};
    s.n = n;
    s.N = n * n;
    s.K = K;
    int off = 0;
    for (int t = 0; t < K; ++t) {
        s.dx[t] = types_xy[2 * t];
        s.dy[t] = types_xy[2 * t + 1];
        s.off[t] = off;
        off += (n - (s.dx[t] < 0 ? -s.dx[t] : s.dx[t])) * (n - s.dy[t]);
    }
    s.off[K] = off;
    s.P = off;
    SolveLaunch L{};
    L.sel = s;
    L.n_units = U;
    L.ci4 = ci4 != 0;
    L.vcache = vcache != 0;
    L.exclusive = false;
    L.lds_bytes = solve_lds_bytes(s, vcache);
    L.o = {iopts[0], iopts[1], iopts[2], iopts[3], iopts[4], fopts[0], fopts[1]};
    L.vred = vred;
    L.gains_in = reinterpret_cast<const float2*>(gains_in);
    L.gains_ref = reinterpret_cast<const float2*>(gains_ref);
    L.gains_out = reinterpret_cast<float2*>(gains_out);
    L.vmodel = reinterpret_cast<float2*>(vmodel);
    L.chisq = chisq;
    L.niter = niter;
    L.status = status;
    std::vector<unsigned char> ldsbuf(L.lds_bytes + 256, 0xCD);
    for (int u = 0; u < U; ++u) {
        bool ok;
        // the same workgroup shapes as the GPU launch; `threads` = 0 picks
        // them by grid size, otherwise it forces one (for the tests)
        const int N = s.N;
        const int nt = threads > 0 ? threads : (N <= 256 ? 256 : (N <= 512 ? 512 : 1024));
        if (nt == 64 && N <= 64) ok = run_shape<64, 1>(L, ldsbuf.data(), u);
        else if (nt == 64 && N <= 128) ok = run_shape<64, 2>(L, ldsbuf.data(), u);
        else if (nt == 64 && N <= 256) ok = run_shape<64, 4>(L, ldsbuf.data(), u);
        else if (nt == 256 && N <= 256) ok = run_shape<256, 1>(L, ldsbuf.data(), u);
        else if (nt == 512 && N <= 512) ok = run_shape<512, 1>(L, ldsbuf.data(), u);
        else if (nt == 1024 && N <= 1024) ok = run_shape<1024, 1>(L, ldsbuf.data(), u);
        else return -1;
        if (!ok) return -2;     // barriers not reached uniformly
    }
    return 0;
}
