// Host shims that let the workgroup bodies of the kernels compile as plain
// C++ (RRC_HOST_EMU).  Every work-item of a workgroup runs as a cooperative
// fiber in one OS thread; __syncthreads() completes once every fiber has
// reached it, and the wave-level exchange behind __shfl_xor once the 64
// fibers of the wave have.  Barriers reached by only some fibers are
// reported as non-uniform.  The order in which the fibers run between two
// barriers is selectable (forward, reverse or a seeded shuffle per
// interval): results that depend on it reveal a data race.  Used only by the
// CPU test-suite to exercise kernel logic without a GPU; the library itself
// never includes this file.
#pragma once

#include <ucontext.h>

#include <cmath>
#include <cstddef>
#include <cstdint>
#include <cstring>
#include <algorithm>
#include <functional>
#include <random>
#include <vector>

#define __host__
#define __device__
#define __forceinline__ inline
#define __align__(x) alignas(x)

struct float2 { float x, y; };
struct double2 { double x, y; };
struct int2 { int x, y; };
struct uint2 { unsigned x, y; };
inline uint2 make_uint2(unsigned a, unsigned b) { return uint2{a, b}; }
struct float4 { float x, y, z, w; };
inline float4 make_float4(float a, float b, float c, float d) { return float4{a, b, c, d}; }
inline float2 make_float2(float a, float b) { return float2{a, b}; }
inline double2 make_double2(double a, double b) { return double2{a, b}; }
inline int2 make_int2(int a, int b) { return int2{a, b}; }

using std::isinf;

inline float __int_as_float(int v) { float f; std::memcpy(&f, &v, 4); return f; }
inline int __float_as_int(float f) { int v; std::memcpy(&v, &f, 4); return v; }

namespace rrc_emu {

struct Dim {
    unsigned x;
};

enum State { RUN = 0, AT_BLOCK = 1, AT_WAVE = 2, DONE = 3 };

struct Group {
    int nthreads = 0;
    std::vector<ucontext_t> ctx;
    std::vector<std::vector<char>> stacks;
    std::vector<int> state;
    ucontext_t sched;
    double xbuf[1024];
    bool bad_barrier = false;
    int order = 0;            // 0 forward, 1 reverse, 2 shuffled per interval
    unsigned seed = 1;
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
    group().state[cur().x] = DONE;
}

inline void wait_as(int st) {
    Group& g = group();
    g.state[cur().x] = st;
    swapcontext(&g.ctx[cur().x], &g.sched);
}

// Runs f() as `nthreads` work-items of one workgroup (waves of 64).
// Work-items run until they reach a barrier; a wave barrier releases when
// all 64 work-items of the wave wait at one, a workgroup barrier when all
// work-items do.  Returns false if the barriers were not reached uniformly.
inline bool run_group(int nthreads, const std::function<void()>& f) {
    Group& g = group();
    g.nthreads = nthreads;
    g.ctx.assign(nthreads, ucontext_t{});
    g.stacks.assign(nthreads, std::vector<char>(256 * 1024));
    g.state.assign(nthreads, RUN);
    g.bad_barrier = false;
    body() = f;
    for (int t = 0; t < nthreads; ++t) {
        getcontext(&g.ctx[t]);
        g.ctx[t].uc_stack.ss_sp = g.stacks[t].data();
        g.ctx[t].uc_stack.ss_size = g.stacks[t].size();
        g.ctx[t].uc_link = &g.sched;
        makecontext(&g.ctx[t], fiber_entry, 0);
    }
    std::vector<int> perm(nthreads);
    for (int t = 0; t < nthreads; ++t) perm[t] = t;
    std::mt19937 rng(g.seed);
    if (g.order == 1) std::reverse(perm.begin(), perm.end());
    const int nwaves = (nthreads + 63) / 64;
    while (true) {
        if (g.order == 2) std::shuffle(perm.begin(), perm.end(), rng);
        for (int q = 0; q < nthreads; ++q) {
            const int t = perm[q];
            if (g.state[t] != RUN) continue;
            cur().x = (unsigned)t;
            swapcontext(&g.sched, &g.ctx[t]);
        }
        // every work-item now waits at a barrier or is done
        bool released = false;
        for (int w = 0; w < nwaves; ++w) {
            int at_wave = 0, done = 0, cnt = 0;
            for (int t = w * 64; t < std::min(nthreads, w * 64 + 64); ++t, ++cnt) {
                at_wave += g.state[t] == AT_WAVE;
                done += g.state[t] == DONE;
            }
            if (at_wave == cnt) {
                for (int t = w * 64; t < w * 64 + cnt; ++t) g.state[t] = RUN;
                released = true;
            } else if (at_wave > 0 && done > 0) {
                g.bad_barrier = true;
                return false;
            }
        }
        if (released) continue;
        int at_block = 0, done = 0;
        for (int t = 0; t < nthreads; ++t) {
            at_block += g.state[t] == AT_BLOCK;
            done += g.state[t] == DONE;
        }
        if (done == nthreads) return true;
        if (at_block == nthreads) {
            for (int t = 0; t < nthreads; ++t) g.state[t] = RUN;
            continue;
        }
        g.bad_barrier = true;      // mixed: some at a barrier the others never reach
        return false;
    }
}

}  // namespace rrc_emu

#define threadIdx (rrc_emu::cur())

inline void __syncthreads() { rrc_emu::wait_as(rrc_emu::AT_BLOCK); }

// Cross-lane exchange within a wave: all 64 work-items of the wave call it
// together.
template <typename T>
inline T __shfl_xor(T v, int o, int /*width*/) {
    rrc_emu::Group& g = rrc_emu::group();
    const unsigned t = rrc_emu::cur().x;
    g.xbuf[t] = (double)v;
    rrc_emu::wait_as(rrc_emu::AT_WAVE);
    const T r = (T)g.xbuf[rrc_emu::cur().x ^ (unsigned)o];
    rrc_emu::wait_as(rrc_emu::AT_WAVE);
    return r;
}
