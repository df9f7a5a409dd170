// Internal interface between the C ABI (pmace_api.hip) and the kernels
// (pmace_kernels.hip).  Not installed; callers use include/pmace.h.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace pmace {

// Device view of one reconstruction.  All pointers live in the caller's
// workspace.
struct DevState {
  float2* t;            // J*Np*Np   t_j = v_j - 2 rho w_j  (v_j = t_j + 2 rho P_j xbar)
  float* ys;            // J*Np*Np   Np*sqrt(z_j)/(1+alpha), DC at [0,0]
  int2* pos;            // J         (row, col) top-left of P_j
  float2* d;            // Np*Np     probe
  float4* pc;           // Np*Np     {Re, Im of d^{-1}/Np^2, |d|^kappa, [d == 0]}
  float* laminv;        // N1*N2     Lambda^{-1} (0 where Lambda = 0)
  float* num;           // N1*N2*2   weighted back-projection accumulator
  float2* xbar;         // N1*N2     consensus image of the last iteration
  float2* xhat;         // N1*N2     reconstruction (Alg. 1 output, kept by recurrence)
  unsigned* status;     // 1 word    bit0: non-finite consensus image; bit1: bad intensity
  float2* stage;        // chunk*Np*Np: Np = 256 spectra being transformed; for every Np
                        // the weighted reflections |d|^kappa (2w - v) the consensus sums
  int2* tiles;          // per gather tile: (start, count) into tile_list
  int* tile_list;       // positions overlapping each tile, ascending
  int n1, n2, np, J;
  float a;              // alpha / (1 + alpha)
  float rho;
  int chunk;            // positions per chunk (all J when Np <= 128)
  const int4* chunk_info;  // host, per chunk: (first tile, tile count, first tile row, tiles per row)
};

// Gather tile of the consensus: GT_R x GT_C object pixels, one thread each.
constexpr int GT_R = 16, GT_C = 64;

// Kernel launchers (stream-ordered; return the hipError_t of the launch).
hipError_t launch_init_amplitudes(const DevState& s, const float* z, float scale, int centered,
                                  hipStream_t st);
hipError_t launch_init_state(const DevState& s, const float2* x0, hipStream_t st);
hipError_t launch_agent(const DevState& s, hipStream_t st);  // one iteration: a2-a9
hipError_t launch_get_state(const DevState& s, float2* v, hipStream_t st);
hipError_t launch_set_state(const DevState& s, const float2* v, hipStream_t st);
hipError_t launch_fft2(int np, int count, const float2* in, float2* out, int inverse, hipStream_t st);

}  // namespace pmace
