// Host-side launch descriptors shared between the C-ABI layer and the
// kernel translation units.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "rrc_device.h"

namespace rrc {

// Geometry tables of a masked lattice (a hexagonal array on its grid),
// rebuilt in the workspace by launch_mask_tables before the kernels that
// read them; every pointer is null for a full square grid.
struct MaskTables {
    const uint8_t* live = nullptr;   // [N] 1 where an antenna sits
    const int* pidx = nullptr;       // [K][N] index of pair (a, a - d_t) in V^reduced, or -1
    const int* pfirst = nullptr;     // [P] first antenna of each pair
    const float* nd = nullptr;       // [2n(n-1)] pairs per lag, V^unique order
    int n_live = 0;                  // antennas
    int ref0 = 0;                    // the first antenna in raster order
};

constexpr int kMaskGridMax = 64;
constexpr int kMaskWords = kMaskGridMax * kMaskGridMax / 32;

struct MaskLaunch {
    Sel sel;                         // the selection, offsets over the mask's pairs
    uint32_t bits[kMaskWords];       // antenna a present: bit a % 32 of word a / 32
    uint8_t* live;
    int* pidx;
    int* pfirst;
    float* nd;
};

struct FftLaunch {
    int M, n, T, n_units;
    int tchunk, nchunk;
    bool ci4;
    const void* volt;
    const float2* gains;
    float* ppart;          // workspace: [U][nchunk][M][M]
    float2* hinv;          // workspace: [U][48][48] 1/g table of the M = 96 kernel (else unused)
    float2* vunique;
    float* vauto;
    unsigned long long* stamps;   // optional [1 + U] run stamps (see unit_done_stamp)
    MaskTables mt;
};

constexpr int kXMaxRuns = 4;   // window runs of the int8-MFMA X-engine's cover

struct XengLaunch {
    Sel sel;
    int T, n_units;
    int tchunk, nchunk;    // time chunks per unit
    int nablk;             // blocks of 256 antennas per unit
    int halo;              // largest raster offset d_t of the selection
    float inv_t;           // 1/T (float outputs)
    bool ci4;
    const void* volt;
    void* vpart;           // workspace: [U][nchunk][P] float2 or int2 (nchunk > 1)
    void* vred;            // output: [U][P] float2 (scaled by 1/T) or int2
    // 4-bit voltages on the int8 matrix cores (xmfma.hip): the instantiation,
    // the runs of 16-antenna column windows (offsets from a row block's first
    // antenna), and the staged antennas of a workgroup [a0 + mf_lo, + mf_cnt)
    bool mfma;
    int mf_inst, mf_nrun, mf_start[kXMaxRuns], mf_len[kXMaxRuns], mf_lo, mf_cnt;
    MaskTables mt;
};

struct SolveOpts {
    int init_mode, degen_mode, max_gn, fp64_steps, max_cg;
    float cg_tol, tol32;
};

struct SolveLaunch {
    Sel sel;
    int n_units;
    bool ci4;
    bool vcache;           // V^reduced copied into LDS beside the state
    bool exclusive;        // one workgroup per CU (at most as many units as CUs)
    size_t lds_bytes;      // dynamic LDS per workgroup
    SolveOpts o;
    const void* vred;
    const float2* gains_in;
    const float2* gains_ref;
    float2* gains_out;
    float2* vmodel;
    float* chisq;
    int* niter;
    int* status;
    unsigned long long* stamps;   // optional [1 + U] run stamps (see unit_done_stamp)
    MaskTables mt;                // a masked lattice's tables (start from the caller's gains)
};

// Damped per-parameter updates (omnical.hip) over the plan's selection or,
// with `all`, every canonical type of the grid in lag order.
struct OmniLaunch {
    int n, K, P, n_units;
    bool all;              // every canonical type (K = 2 n (n - 1)), lag order
    bool ci4;              // V^reduced as raw int32 sums
    Sel sel;               // the selection when !all
    size_t lds_types;      // LDS bytes of the every-type table (0 when !all)
    int max_iter;
    float tol, damping;
    bool finish;           // fix the degeneracies and compute chi^2 at exit
    const float2* gains_in;    // start (V from the group means), or null: continue
    const void* vred;
    void* gains;           // [U][N] state and output
    void* vmodel;          // [U][K] state and output
    float* chisq;
    int* niter;
    int* status;
    float* delta;          // optional [U]: the last relative change
    MaskTables mt;         // a masked lattice's tables (selection only)
};

// Low-cadence X-engine (lowcad.hip): every pair of an n x n grid, each
// integrated over the samples of its cycle.
constexpr int kLowcadMaxCycles = 256;
struct LowcadLaunch {
    int n, n_units, T, n_cycles;
    int type_begin[kLowcadMaxCycles + 1];   // cycle c = lag-order types [type_begin[c], type_begin[c+1])
    const void* volt;      // [U][T][N] complex64
    void* vfull;           // [U][N (N - 1) / 2] complex64, the all-type pair list
};

struct ChisqLaunch {
    Sel sel;
    int n_units;
    const float2* g;
    const float2* vm;
    const float2* vred;
    float* chisq;
    float2* grad_g;
    float2* grad_v;
    float* diag_g;
    float* diag_v;
};

#ifndef RRC_HOST_EMU
int fft_samples_per_step_for(int M);
hipError_t launch_fftcorr(const FftLaunch& L, hipStream_t st);
hipError_t launch_xengine(const XengLaunch& L, hipStream_t st);
size_t xengine_lds_bytes(int halo, bool ci4);
int xengine_antennas_per_block(bool ci4);
int xengine_max_halo();
int xengine_samples_per_step(bool ci4);
bool xmfma_plan(const Sel& s, XengLaunch& X);
hipError_t launch_xmfma(const XengLaunch& X, hipStream_t st);
size_t solve_lds_bytes(const Sel& s, bool vcache);
hipError_t prepare_solve(const SolveLaunch& L);
hipError_t launch_solve(const SolveLaunch& L, hipStream_t st);
hipError_t launch_chisq(const ChisqLaunch& L, hipStream_t st, bool adjoint);
hipError_t launch_omnical(const OmniLaunch& L, hipStream_t st);
hipError_t launch_xlowcad(const LowcadLaunch& L, hipStream_t st);
size_t omnical_lds_bytes(int n, int K, bool all);
int omnical_max_all_grid();
hipError_t launch_stamp_start(unsigned long long* stamps, int n_units, hipStream_t st);
hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t st);
hipError_t launch_mask_tables(const MaskLaunch& L, hipStream_t st);
#endif

}  // namespace rrc
