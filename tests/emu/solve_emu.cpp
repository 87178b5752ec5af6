// CPU build of the solver kernel's workgroup body (one std::thread per
// work-item), exposed with a C interface for the host-side test-suite.
#define RRC_HOST_EMU
#include "../../paper_2005_03060_amd/csrc/solve.hip"

#include <vector>

using namespace rrc;

template <int APT>
static bool run_unit(const SolveLaunch& L, bool lds, unsigned char* ldsbuf, int unit) {
    Shared sh;
    return rrc_emu::run_group(kSThreads, [&] {
        if (lds) solve_unit<APT, true>(L, sh, ldsbuf, unit);
        else solve_unit<APT, false>(L, sh, ldsbuf, unit);
    });
}

extern "C" int rrc_emu_solve(int n, const int* types_xy, int K, int U, int ci4, const void* vred,
                             const void* gains_in, const void* gains_ref, const int* iopts,
                             const float* fopts, void* gains_out, void* vmodel, float* chisq,
                             int* niter, int* status, int use_lds, int order) {
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
    L.lds = use_lds != 0;
    L.lds_bytes = solve_lds_bytes(s, L.lds);
    L.slab_bytes = (solve_slab_bytes(s, L.lds) + 255) & ~(size_t)255;
    L.o = {iopts[0], iopts[1], iopts[2], iopts[3], iopts[4], fopts[0], fopts[1]};
    L.vred = vred;
    L.gains_in = reinterpret_cast<const float2*>(gains_in);
    L.gains_ref = reinterpret_cast<const float2*>(gains_ref);
    L.gains_out = reinterpret_cast<float2*>(gains_out);
    L.vmodel = reinterpret_cast<float2*>(vmodel);
    L.chisq = chisq;
    L.niter = niter;
    L.status = status;
    std::vector<unsigned char> slab((size_t)U * L.slab_bytes + 256, 0xAB);
    std::vector<unsigned char> ldsbuf(L.lds_bytes + 256, 0xCD);
    L.slab = reinterpret_cast<char*>(slab.data());
    const int apt = (s.N + kSThreads - 1) / kSThreads;
    for (int u = 0; u < U; ++u) {
        bool ok;
        if (apt <= 1) ok = run_unit<1>(L, L.lds, ldsbuf.data(), u);
        else if (apt <= 2) ok = run_unit<2>(L, L.lds, ldsbuf.data(), u);
        else if (apt <= 4) ok = run_unit<4>(L, L.lds, ldsbuf.data(), u);
        else return -1;
        if (!ok) return -2;     // barriers not reached uniformly
    }
    return 0;
}
