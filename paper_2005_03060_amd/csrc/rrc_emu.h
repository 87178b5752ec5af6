// Host shims that let the workgroup bodies of the kernels compile as plain
// C++ (RRC_HOST_EMU).  Every work-item of a workgroup runs as a cooperative
// fiber in one OS thread; __syncthreads() switches to the next fiber, so a
// barrier completes once every fiber has reached it.  __shfl_xor goes
// through a shared exchange buffer between two barriers.  A fiber that
// finishes while others still wait at a barrier is reported as a
// non-uniform barrier.  Used only by the CPU test-suite to exercise kernel
// logic without a GPU; the library itself never includes this file.
#pragma once

#include <ucontext.h>

#include <cmath>
#include <cstddef>
#include <cstdint>
#include <functional>
#include <vector>

#define __host__
#define __device__
#define __forceinline__ inline
#define __align__(x) alignas(x)

struct float2 { float x, y; };
struct double2 { double x, y; };
struct int2 { int x, y; };
inline float2 make_float2(float a, float b) { return float2{a, b}; }
inline double2 make_double2(double a, double b) { return double2{a, b}; }
inline int2 make_int2(int a, int b) { return int2{a, b}; }

using std::isinf;

namespace rrc_emu {

struct Dim {
    unsigned x;
};

struct Group {
    int nthreads = 0;
    std::vector<ucontext_t> ctx;
    std::vector<std::vector<char>> stacks;
    std::vector<char> done;
    ucontext_t sched;
    double xbuf[1024];
    bool bad_barrier = false;
};

inline Group& group() {
    static Group g;
    return g;
}
inline Dim& cur() {
    static Dim d{0};
    return d;
}
inline std::function<void()>& body() {
    static std::function<void()> f;
    return f;
}

inline void fiber_entry() {
    body()();
    group().done[cur().x] = 1;
}

// Runs f() as `nthreads` work-items of one workgroup.  Returns false if the
// barriers were not reached uniformly.
inline bool run_group(int nthreads, const std::function<void()>& f) {
    Group& g = group();
    g.nthreads = nthreads;
    g.ctx.assign(nthreads, ucontext_t{});
    g.stacks.assign(nthreads, std::vector<char>(256 * 1024));
    g.done.assign(nthreads, 0);
    g.bad_barrier = false;
    body() = f;
    for (int t = 0; t < nthreads; ++t) {
        getcontext(&g.ctx[t]);
        g.ctx[t].uc_stack.ss_sp = g.stacks[t].data();
        g.ctx[t].uc_stack.ss_size = g.stacks[t].size();
        g.ctx[t].uc_link = &g.sched;
        makecontext(&g.ctx[t], fiber_entry, 0);
    }
    while (true) {
        int finished = 0;
        for (int t = 0; t < nthreads; ++t) {
            if (g.done[t]) {
                ++finished;
                continue;
            }
            cur().x = (unsigned)t;
            swapcontext(&g.sched, &g.ctx[t]);
            if (g.done[t]) ++finished;
        }
        if (finished == nthreads) break;
        if (finished > 0) {            // some returned while others wait at a barrier
            g.bad_barrier = true;
            break;
        }
    }
    return !g.bad_barrier;
}

}  // namespace rrc_emu

#define threadIdx (rrc_emu::cur())

inline void __syncthreads() {
    rrc_emu::Group& g = rrc_emu::group();
    swapcontext(&g.ctx[rrc_emu::cur().x], &g.sched);
}

// All work-items of the group call this together (uniform control flow).
template <typename T>
inline T __shfl_xor(T v, int o, int /*width*/) {
    rrc_emu::Group& g = rrc_emu::group();
    const unsigned t = rrc_emu::cur().x;
    g.xbuf[t] = (double)v;
    __syncthreads();
    const T r = (T)g.xbuf[rrc_emu::cur().x ^ (unsigned)o];
    __syncthreads();
    return r;
}
