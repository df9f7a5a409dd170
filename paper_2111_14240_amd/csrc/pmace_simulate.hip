// Simulated ptychographic measurements on the GPU (Sec. II eq. (1) and
// Sec. IV eq. (16)):
//     I_j = |F D P_j x|^2                       (noise-free intensities)
//     z_j = Pois(I_j * r_p / max_{j,k} I_j[k])  (peak photon rate r_p)
// The maximum is taken over every position and pixel (one scale for the
// whole experiment).  Random numbers come from a counter-based generator,
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
// easy as 1, 2, 3", SC 2011), keyed by the seed and counted by element index,
// so every sample is reproducible and independent of the launch shape.
// Poisson variates: the product-of-uniforms method below mean 10, and
// Hormann's transformed rejection with squeeze (PTRS; W. Hormann, "The
// transformed rejection method for generating Poisson random variables",
// Insurance: Mathematics and Economics 12, 1993) from mean 10 up.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <new>

#include "pmace.h"
#include "pmace_dft.hpp"
#include "pmace_internal.hpp"

namespace pmace {

// ---------------------------------------------------------------------------
// Philox4x32-10: ten rounds of two 32x32->64 multiplies, a xor with the key,
// and a Weyl increment of the key between rounds.
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint2 k) {
  const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
  const uint32_t w0 = 0x9E3779B9u, w1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(m0, c.x), lo0 = m0 * c.x;
    const uint32_t hi1 = __umulhi(m1, c.z), lo1 = m1 * c.z;
    c = make_uint4(hi1 ^ c.y ^ k.x, lo1, hi0 ^ c.w ^ k.y, lo0);
    k.x += w0;
    k.y += w1;
  }
  return c;
}

// Uniform doubles in (0, 1) for element `idx`: block n of the stream is
// Philox(counter = (idx lo, idx hi, n, 0x50495853), key = seed).
struct Uniforms {
  uint2 key;
  uint32_t i0, i1, n;
  uint4 buf;
  int have;
  __device__ Uniforms(uint64_t seed, uint64_t idx)
      : key(make_uint2((uint32_t)seed, (uint32_t)(seed >> 32))),
        i0((uint32_t)idx), i1((uint32_t)(idx >> 32)), n(0), have(0) {}
  __device__ double next() {
    if (have == 0) {
      buf = philox4x32_10(make_uint4(i0, i1, n++, 0x50495853u), key);
      have = 2;
    }
    const uint32_t a = have == 2 ? buf.x : buf.z, b = have == 2 ? buf.y : buf.w;
    --have;
    // 53 random bits, centred in their interval: never 0 or 1
    return ((double)(a >> 5) * 67108864.0 + (double)(b >> 6) + 0.5) * (1.0 / 9007199254740992.0);
  }
};

__device__ double poisson_draw(double lam, Uniforms& u) {
  if (!(lam > 0.0)) return 0.0;
  if (lam < 10.0) {
    const double L = exp(-lam);
    double p = 1.0;
    int k = 0;
    do {
      ++k;
      p *= u.next();
    } while (p > L && k < 1000);
    return (double)(k - 1);
  }
  const double slam = sqrt(lam), loglam = log(lam);
  const double b = 0.931 + 2.53 * slam;
  const double a = -0.059 + 0.02483 * b;
  const double invalpha = 1.1239 + 1.1328 / (b - 3.4);
  const double vr = 0.9277 - 3.6224 / (b - 2.0);
  for (int it = 0; it < 1000; ++it) {  // each try accepts with probability > 0.8
    const double U = u.next() - 0.5;
    const double V = u.next();
    const double us = 0.5 - fabs(U);
    const double k = floor((2.0 * a / us + b) * U + lam + 0.43);
    if (us >= 0.07 && V <= vr) return k;
    if (k < 0.0 || (us < 0.013 && V > us)) continue;
    if (log(V) + log(invalpha) - log(a / (us * us) + b) <= -lam + k * loglam - lgamma(k + 1.0))
      return k;
  }
  return floor(lam + 0.5);
}

// ---------------------------------------------------------------------------
// Noise-free intensities I_j = |F D P_j x|^2 (F orthonormal) and their
// maximum, with the frames d P_j x formed as the transform loads them and the
// intensities as it stores them.  The maximum is folded per workgroup into
// one atomic (non-negative floats order as their bit patterns, so an
// unsigned max is a float max).
// ---------------------------------------------------------------------------
constexpr int kSimRB = PMACE_RB;   // rows per workgroup of the row pass (Np > 128)
constexpr int kSimCB = PMACE_CB;   // columns per workgroup of the column pass
static_assert(160 % kSimRB == 0 && 192 % kSimRB == 0 && 256 % kSimRB == 0, "row block");
static_assert(160 % kSimCB == 0 && 192 % kSimCB == 0 && 256 % kSimCB == 0, "column block");

template <int NT>
__device__ __forceinline__ void block_max_to(float v, unsigned* maxbits) {
  static_assert(NT % 64 == 0 && NT <= 1024, "whole wavefronts");
  __shared__ float wmax[NT / 64];
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < NT / 64; ++w) v = fmaxf(v, wmax[w]);
    atomicMax(maxbits, __float_as_uint(v));
  }
}

// Np <= 128: one position per workgroup, the whole frame in LDS.
template <int NP>
__global__ void __launch_bounds__(NP * Geo<NP>::A)
sim_small_k(const float2* __restrict__ d, const int2* __restrict__ pos, const float2* __restrict__ x,
            int n2, float* __restrict__ z, unsigned* __restrict__ maxbits) {
  constexpr int A = Geo<NP>::A, B = Geo<NP>::B, S = NP + A, NT = NP * A, M = B / A;
  static_assert(exch_phases<NP>() == 1, "the whole-frame tile exchanges in one round");
  __shared__ float2 tile[NP * S];
  __shared__ float2 tw[NP];
  const int tid = threadIdx.x;
  fill_twiddles<NP>(tw, tid, NT);
  const int j = blockIdx.x;
  const int2 pj = pos[j];
  const int r = tid / A, p = tid % A, c = tid % NP, q = tid / NP;
  const float2* xrow = x + (size_t)(pj.x + r) * n2 + pj.y;
  float2* row = tile + r * S;
  float2 v[B];
#pragma unroll
  for (int nb = 0; nb < B; ++nb) {
    const int cc = p + A * nb;
    v[nb] = cmul(d[r * NP + cc], xrow[cc]);
  }
  __syncthreads();
  row_fwd<NP>(v, row, p, tw);
  __syncthreads();
#pragma unroll
  for (int m = 0; m < M; ++m)
#pragma unroll
    for (int ka = 0; ka < A; ++ka) row[p + A * m + B * ka] = v[m * A + ka];
  __syncthreads();
#pragma unroll
  for (int nb = 0; nb < B; ++nb) v[nb] = tile[(q + A * nb) * S + c];
  col_fwd<NP>(v, tile, S, c, q, tw);
  const float scale = 1.f / NP;
  float* zj = z + (size_t)j * NP * NP;
  float mx = 0.f;
#pragma unroll
  for (int m = 0; m < M; ++m)
#pragma unroll
    for (int ka = 0; ka < A; ++ka) {
      const float2 s = cscale(v[m * A + ka], scale);
      const float e = fmaf(s.x, s.x, s.y * s.y);
      zj[(size_t)(q + A * m + B * ka) * NP + c] = e;
      mx = fmaxf(mx, e);
    }
  block_max_to<NT>(mx, maxbits);
}

// Np > 128, row pass: frames and forward row DFTs (scaled 1/sqrt(Np)) to fr.
template <int NP>
__global__ void __launch_bounds__(kSimRB * Geo<NP>::A)
sim_rows_k(const float2* __restrict__ d, const int2* __restrict__ pos, const float2* __restrict__ x,
           int n2, float2* __restrict__ fr, float sc) {
  constexpr int A = Geo<NP>::A, B = Geo<NP>::B, M = B / A, S = row_cap<NP>();
  __shared__ float2 tile[kSimRB * S];
  __shared__ float2 tw[NP];
  const int tid = threadIdx.x;
  fill_twiddles<NP>(tw, tid, kSimRB * A);
  const int j = blockIdx.x / (NP / kSimRB), rb = blockIdx.x % (NP / kSimRB);
  const int rl = tid / A, p = tid % A, r = rb * kSimRB + rl;
  const int2 pj = pos[j];
  const float2* xrow = x + (size_t)(pj.x + r) * n2 + pj.y;
  float2 v[B];
#pragma unroll
  for (int nb = 0; nb < B; ++nb) {
    const int cc = p + A * nb;
    v[nb] = cmul(d[r * NP + cc], xrow[cc]);
  }
  __syncthreads();
  row_fwd<NP>(v, tile + rl * S, p, tw);
  float2* out = fr + ((size_t)j * NP + r) * NP;
#pragma unroll
  for (int m = 0; m < M; ++m)
#pragma unroll
    for (int ka = 0; ka < A; ++ka) out[p + A * m + B * ka] = cscale(v[m * A + ka], sc);
}

// Np > 128, column pass: forward column DFTs (scaled 1/sqrt(Np)) and the
// intensities.
template <int NP>
__global__ void __launch_bounds__(kSimCB * Geo<NP>::A)
sim_cols_k(const float2* __restrict__ fr, float* __restrict__ z, unsigned* __restrict__ maxbits, float sc) {
  constexpr int A = Geo<NP>::A, B = Geo<NP>::B, M = B / A, NT = kSimCB * A;
  __shared__ float2 tile[col_rows<NP>() * kSimCB];
  __shared__ float2 tw[NP];
  const int tid = threadIdx.x;
  fill_twiddles<NP>(tw, tid, NT);
  const int j = blockIdx.x / (NP / kSimCB), cb = blockIdx.x % (NP / kSimCB);
  const int c = tid % kSimCB, q = tid / kSimCB, col = cb * kSimCB + c;
  const size_t base = (size_t)j * NP * NP + col;
  float2 v[B];
#pragma unroll
  for (int nb = 0; nb < B; ++nb) v[nb] = fr[base + (size_t)(q + A * nb) * NP];
  __syncthreads();
  col_fwd<NP>(v, tile, kSimCB, c, q, tw);
  float mx = 0.f;
#pragma unroll
  for (int m = 0; m < M; ++m)
#pragma unroll
    for (int ka = 0; ka < A; ++ka) {
      const float2 s = cscale(v[m * A + ka], sc);
      const float e = fmaf(s.x, s.x, s.y * s.y);
      z[base + (size_t)(q + A * m + B * ka) * NP] = e;
      mx = fmaxf(mx, e);
    }
  block_max_to<NT>(mx, maxbits);
}

template <int NP>
hipError_t launch_sim_intensities(int J, const float2* d, const int2* pos, const float2* x, int n2,
                                  float2* fr, float* z, unsigned* maxbits, hipStream_t st) {
  if constexpr (NP <= 128) {
    hipLaunchKernelGGL(sim_small_k<NP>, dim3(J), dim3(NP * Geo<NP>::A), 0, st, d, pos, x, n2, z, maxbits);
  } else {
    const float sc = 1.f / sqrtf((float)NP);  // 1/sqrt(Np) per pass
    hipLaunchKernelGGL(sim_rows_k<NP>, dim3(J * (NP / kSimRB)), dim3(kSimRB * Geo<NP>::A), 0, st, d, pos,
                       x, n2, fr, sc);
    hipLaunchKernelGGL(sim_cols_k<NP>, dim3(J * (NP / kSimCB)), dim3(kSimCB * Geo<NP>::A), 0, st, fr, z,
                       maxbits, sc);
  }
  return hipGetLastError();
}

__global__ void poisson_k(float* __restrict__ z, const unsigned* __restrict__ maxbits, double peak,
                          uint64_t seed, long long total) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const double mx = (double)__uint_as_float(*maxbits);
  const double scale = mx > 0.0 ? peak / mx : 0.0;
  Uniforms u(seed, (uint64_t)i);
  z[i] = (float)poisson_draw((double)z[i] * scale, u);
}

__global__ void philox_k(uint32_t* io, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t* r = io + 6 * (size_t)i;
  const uint4 o = philox4x32_10(make_uint4(r[0], r[1], r[2], r[3]), make_uint2(r[4], r[5]));
  r[0] = o.x;
  r[1] = o.y;
  r[2] = o.z;
  r[3] = o.w;
}

__global__ void poisson_test_k(const double* __restrict__ lam, float* __restrict__ out, uint64_t seed,
                               int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  Uniforms u(seed, (uint64_t)i);
  out[i] = (float)poisson_draw(lam[i], u);
}

// Clears the maximum and the position flag (a kernel, not a memset, so the
// call stays capturable).
__global__ void sim_clear_k(unsigned* __restrict__ ctl) {
  if (threadIdx.x < 2) ctl[threadIdx.x] = 0u;
}

// Flags (ctl[1] = 1) any position whose patch leaves the object.
__global__ void sim_check_pos_k(const int2* __restrict__ pos, int J, int n1, int n2, int np,
                                unsigned* __restrict__ ctl) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= J) return;
  const int2 p = pos[j];
  if (p.x < 0 || p.y < 0 || p.x > n1 - np || p.y > n2 - np) atomicOr(ctl + 1, 1u);
}

// Scratch of the allocation-free entry point: the maximum and the position
// flag in the first 256 bytes, then (Np > 128) the frames' row transforms.
// One copy per device, held until the process ends.
constexpr size_t kSimScratchBytes = (size_t)64 << 20;
__device__ __align__(256) unsigned char scratch[kSimScratchBytes];

}  // namespace pmace

namespace {
inline unsigned nblocks(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }
inline size_t up256(size_t x) { return (x + 255) & ~(size_t)255; }

// Intensities, optional Poisson draws and the scale, into z_d; `fr` holds the
// row transforms (Np > 128), `maxbits` the cleared maximum.  Stream-ordered;
// synchronises only to return the scale.
pmace_status run_simulation(int32_t n2, int32_t np, int32_t num_pos, const void* probe_d,
                            const int32_t* pos_d, const void* x_d, double peak_photons, uint64_t seed,
                            float* z_d, float2* fr, unsigned* maxbits, double* scale_out,
                            hipStream_t st) {
  const long long total = (long long)num_pos * np * np;
  const float2* dd = reinterpret_cast<const float2*>(probe_d);
  const int2* pp = reinterpret_cast<const int2*>(pos_d);
  const float2* xx = reinterpret_cast<const float2*>(x_d);
  hipError_t e = hipErrorInvalidValue;
  switch (np) {
    case 32: e = pmace::launch_sim_intensities<32>(num_pos, dd, pp, xx, n2, fr, z_d, maxbits, st); break;
    case 48: e = pmace::launch_sim_intensities<48>(num_pos, dd, pp, xx, n2, fr, z_d, maxbits, st); break;
    case 64: e = pmace::launch_sim_intensities<64>(num_pos, dd, pp, xx, n2, fr, z_d, maxbits, st); break;
    case 96: e = pmace::launch_sim_intensities<96>(num_pos, dd, pp, xx, n2, fr, z_d, maxbits, st); break;
    case 128: e = pmace::launch_sim_intensities<128>(num_pos, dd, pp, xx, n2, fr, z_d, maxbits, st); break;
    case 160: e = pmace::launch_sim_intensities<160>(num_pos, dd, pp, xx, n2, fr, z_d, maxbits, st); break;
    case 192: e = pmace::launch_sim_intensities<192>(num_pos, dd, pp, xx, n2, fr, z_d, maxbits, st); break;
    case 256: e = pmace::launch_sim_intensities<256>(num_pos, dd, pp, xx, n2, fr, z_d, maxbits, st); break;
    default: break;
  }
  if (e != hipSuccess) return PMACE_EDEVICE;
  if (peak_photons > 0.0)
    hipLaunchKernelGGL(pmace::poisson_k, dim3(nblocks(total, 256)), dim3(256), 0, st, z_d, maxbits,
                       peak_photons, seed, total);
  if (hipGetLastError() != hipSuccess) return PMACE_EDEVICE;
  if (scale_out) {
    unsigned mb = 0;
    if (hipMemcpyAsync(&mb, maxbits, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return PMACE_EDEVICE;
    float mx;
    std::memcpy(&mx, &mb, 4);
    *scale_out = (peak_photons > 0.0 && mx > 0.f) ? peak_photons / (double)mx : 1.0;
  }
  return PMACE_OK;
}


// Device address of `scratch` on each device, looked up once per device.
std::mutex g_scratch_mu;
void* g_scratch_ptr[64] = {};

unsigned char* scratch_of_current_device() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(pmace::scratch)) != hipSuccess || !p) return nullptr;
    g_scratch_ptr[dev] = p;
  }
  return static_cast<unsigned char*>(g_scratch_ptr[dev]);
}
}  // namespace

extern "C" {

size_t pmace_simulate_footprint(int32_t np, int32_t num_pos) {
  if (np < 1 || num_pos < 1) return 0;
  return up256((size_t)num_pos * np * np * 8) + 256 + 256;
}

pmace_status pmace_simulate(int32_t n1, int32_t n2, int32_t np, int32_t num_pos, const void* probe_d,
                            const int32_t* pos_d, const void* x_d, double peak_photons,
                            uint64_t seed, float* z_d, void* workspace_d, size_t ws_bytes,
                            double* scale_out, void* hip_stream) {
  if (np < 1 || num_pos < 1 || n1 < np || n2 < np || !probe_d || !pos_d || !x_d || !z_d ||
      !workspace_d || !std::isfinite(peak_photons))
    return PMACE_EINVAL;
  if (np != 32 && np != 48 && np != 64 && np != 96 && np != 128 && np != 160 && np != 192 && np != 256)
    return PMACE_EUNSUPPORTED;
  if (ws_bytes < pmace_simulate_footprint(np, num_pos)) return PMACE_ENOMEM;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  // positions are checked on the host: the frame gather reads the object there
  const size_t J = (size_t)num_pos;
  int32_t* pos = new (std::nothrow) int32_t[2 * J];
  if (!pos) return PMACE_ENOMEM;
  if (hipMemcpyAsync(pos, pos_d, J * 8, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess) {
    delete[] pos;
    return PMACE_EDEVICE;
  }
  bool ok = true;
  for (size_t j = 0; j < J; ++j)
    if (pos[2 * j] < 0 || pos[2 * j + 1] < 0 || pos[2 * j] > n1 - np || pos[2 * j + 1] > n2 - np) ok = false;
  delete[] pos;
  if (!ok) return PMACE_EINVAL;

  char* base = reinterpret_cast<char*>(up256(reinterpret_cast<size_t>(workspace_d)));
  float2* fr = reinterpret_cast<float2*>(base);
  unsigned* maxbits = reinterpret_cast<unsigned*>(base + up256(J * np * np * 8));
  if (hipMemsetAsync(maxbits, 0, 4, st) != hipSuccess) return PMACE_EDEVICE;
  return run_simulation(n2, np, num_pos, probe_d, pos_d, x_d, peak_photons, seed, z_d, fr, maxbits,
                        scale_out, st);
}

size_t pmace_simulate_static_max_bytes(void) { return pmace::kSimScratchBytes - 256; }

pmace_status pmace_simulate_static(int32_t n1, int32_t n2, int32_t np, int32_t num_pos,
                                   const void* probe_d, const int32_t* pos_d, const void* x_d,
                                   double peak_photons, uint64_t seed, float* z_d, double* scale_out,
                                   void* hip_stream) {
  if (np < 1 || num_pos < 1 || n1 < np || n2 < np || !probe_d || !pos_d || !x_d || !z_d ||
      !std::isfinite(peak_photons))
    return PMACE_EINVAL;
  if (np != 32 && np != 48 && np != 64 && np != 96 && np != 128 && np != 160 && np != 192 && np != 256)
    return PMACE_EUNSUPPORTED;
  // Np > 128 keeps every frame's row transform in the scratch array
  const size_t frames = np > 128 ? (size_t)num_pos * np * np * 8 : 0;
  if (frames > pmace_simulate_static_max_bytes()) return PMACE_ENOMEM;
  unsigned char* sp = scratch_of_current_device();
  if (!sp) return PMACE_EDEVICE;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);
  unsigned* ctl = reinterpret_cast<unsigned*>(sp);  // [0] maximum bits, [1] position flag
  float2* fr = reinterpret_cast<float2*>(sp + 256);
  // positions are checked on the device (no host buffer): the frame gather
  // reads the object there, so nothing is launched until they are known good
  hipLaunchKernelGGL(pmace::sim_clear_k, dim3(1), dim3(64), 0, st, ctl);
  hipLaunchKernelGGL(pmace::sim_check_pos_k, dim3(nblocks(num_pos, 256)), dim3(256), 0, st,
                     reinterpret_cast<const int2*>(pos_d), num_pos, n1, n2, np, ctl);
  unsigned bad = 0;
  if (hipGetLastError() != hipSuccess ||
      hipMemcpyAsync(&bad, ctl + 1, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return PMACE_EDEVICE;
  if (bad) return PMACE_EINVAL;
  return run_simulation(n2, np, num_pos, probe_d, pos_d, x_d, peak_photons, seed, z_d, fr, ctl,
                        scale_out, st);
}

pmace_status pmace_philox4x32_10(uint32_t* io_d, int32_t n, void* hip_stream) {
  if (!io_d || n < 0) return PMACE_EINVAL;
  if (n == 0) return PMACE_OK;
  hipLaunchKernelGGL(pmace::philox_k, dim3(nblocks(n, 256)), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(hip_stream), io_d, n);
  return hipGetLastError() == hipSuccess ? PMACE_OK : PMACE_EDEVICE;
}

pmace_status pmace_poisson(const double* lam_d, float* out_d, int32_t n, uint64_t seed,
                           void* hip_stream) {
  if (!lam_d || !out_d || n < 0) return PMACE_EINVAL;
  if (n == 0) return PMACE_OK;
  hipLaunchKernelGGL(pmace::poisson_test_k, dim3(nblocks(n, 256)), dim3(256), 0,
                     reinterpret_cast<hipStream_t>(hip_stream), lam_d, out_d, seed, n);
  return hipGetLastError() == hipSuccess ? PMACE_OK : PMACE_EDEVICE;
}

}  // extern "C"
