// PMACE iteration kernels for gfx950 (MI355X).
//
// One iteration of Alg. 1 is carried as
//     v_j   = t_j + 2 rho P_j xbar                      (finishes line 5 of the previous pass)
//     w_j   = F_j(v_j)                                  (eq. (9), line 3)
//     u_j   = 2 w_j - v_j                               (reflection, line 4)
//     t_j  <- v_j - 2 rho w_j                           (first half of line 5)
//     num  += P_j^t |d|^kappa u_j                       (numerator of eq. (11))
// followed by  xbar = Lambda^{-1} num  and  xhat <- (1-rho) xhat + rho xbar.
// Storing t instead of v is exact algebra of line 5 (v_new = t + 2 rho P_j xbar),
// and the xhat recurrence is exact algebra of the returned weighted average
// (the average of P_j xbar is xbar on covered pixels; the average of w is the
// mean of the averages of u and v).  Each agent state is read and written once
// per iteration.
//
// The agent applies eq. (9) in the Fourier domain: with W = F(d v),
//     F(d w) = W (alpha + y/|W|) / (1 + alpha)   (0 where W = 0)
// which is the r* of eq. (8) with the phase of W, so w = d^{-1} F^*(...) needs
// one forward and one inverse 2-D DFT per patch.  Where d = 0, eq. (6) leaves
// v free and the agent returns its input there.
#include "pmace_dft.hpp"
#include "pmace_internal.hpp"

namespace pmace {

// -------------------------------------------------------------------------
// helpers
// -------------------------------------------------------------------------

__device__ __forceinline__ float2 ldg2(const float2* p) { return *p; }

// Fourier-domain prox of eq. (9): U = W * (a + ys / |W|), 0 where W == 0.
__device__ __forceinline__ float2 fourier_prox(float2 W, float ysv, float a) {
  const float m2 = W.x * W.x + W.y * W.y;
  const float rs = m2 > 0.f ? __builtin_amdgcn_rsqf(m2) : 0.f;
  const float g = fmaf(ysv, rs, a);
  return make_float2(W.x * g, W.y * g);
}

// State update and consensus contribution for one pixel (a6-a8): w from the
// inverse transform z (d^{-1} and the 1/Np^2 folded into pcf.xy; w = v where
// d == 0), t <- v - 2 rho w, and the weighted reflection |d|^kappa (2w - v).
__device__ __forceinline__ void finish_pixel(float2 z, float2 v, float4 pcf, float two_rho,
                                             float2* t_out, float2* u_out) {
  float2 w = cmul(make_float2(pcf.x, pcf.y), z);
  w.x = fmaf(pcf.w, v.x, w.x);
  w.y = fmaf(pcf.w, v.y, w.y);
  *t_out = make_float2(fmaf(-two_rho, w.x, v.x), fmaf(-two_rho, w.y, v.y));
  *u_out = make_float2(pcf.z * (2.f * w.x - v.x), pcf.z * (2.f * w.y - v.y));
}

struct AgentArgs {
  float2* t;
  const float* ys;
  const int2* pos;
  const float2* d;
  const float4* pc;
  const float2* xbar;
  float* num;
  float2* stage;
  int n2;
  float a;
  float two_rho;
  int j0;
};

// -------------------------------------------------------------------------
// Np <= 128: the whole patch lives in LDS; one workgroup per position does
// a2-a8 in one pass (rows, columns, prox, columns, rows, epilogue).
// -------------------------------------------------------------------------
template <int NP>
__global__ void __launch_bounds__(NP * Geo<NP>::A) agent_fused(AgentArgs g) {
  constexpr int A = Geo<NP>::A, B = Geo<NP>::B, S = NP + A, NT = NP * A, M = B / A;
  __shared__ float2 tile[NP * S];
  __shared__ float2 tw[NP];
  const int tid = threadIdx.x;
  fill_twiddles<NP>(tw, tid, NT);
  const int j = g.j0 + blockIdx.x;
  const int2 pj = g.pos[j];
  const size_t pb = (size_t)j * NP * NP;
  const int r = tid / A, p = tid % A;
  const float2* xrow = g.xbar + (size_t)(pj.x + r) * g.n2 + pj.y;
  float2* trow = g.t + pb + (size_t)r * NP;

  float2 x[B];
#pragma unroll
  for (int nb = 0; nb < B; ++nb) {
    const int c = p + A * nb;
    const float2 tt = trow[c];
    const float2 xb = xrow[c];
    const float2 v = make_float2(fmaf(g.two_rho, xb.x, tt.x), fmaf(g.two_rho, xb.y, tt.y));
    x[nb] = cmul(g.d[r * NP + c], v);
  }
  __syncthreads();
  float2* row = tile + r * S;
  row_fwd<NP>(x, row, p, tw);
  __syncthreads();
#pragma unroll
  for (int m = 0; m < M; ++m)
#pragma unroll
    for (int ka = 0; ka < A; ++ka) row[p + A * m + B * ka] = x[m * A + ka];
  __syncthreads();

  const int c = tid % NP, q = tid / NP;
#pragma unroll
  for (int nb = 0; nb < B; ++nb) x[nb] = tile[(q + A * nb) * S + c];
  col_fwd<NP>(x, tile, S, c, q, tw);
  const float* yc = g.ys + pb + c;
#pragma unroll
  for (int m = 0; m < M; ++m)
#pragma unroll
    for (int ka = 0; ka < A; ++ka) {
      const int k = q + A * m + B * ka;
      x[m * A + ka] = fourier_prox(x[m * A + ka], yc[(size_t)k * NP], g.a);
    }
  col_inv<NP>(x, tile, S, c, q, tw);
  __syncthreads();
#pragma unroll
  for (int nb = 0; nb < B; ++nb) tile[(q + A * nb) * S + c] = x[nb];
  __syncthreads();

#pragma unroll
  for (int m = 0; m < M; ++m)
#pragma unroll
    for (int ka = 0; ka < A; ++ka) x[m * A + ka] = row[p + A * m + B * ka];
  row_inv<NP>(x, row, p, tw);

  float2* urow = g.stage + pb + (size_t)r * NP;
#pragma unroll
  for (int nb = 0; nb < B; ++nb) {
    const int cc = p + A * nb;
    const float2 tt = trow[cc];
    const float2 xb = xrow[cc];
    const float2 v = make_float2(fmaf(g.two_rho, xb.x, tt.x), fmaf(g.two_rho, xb.y, tt.y));
    finish_pixel(x[nb], v, g.pc[r * NP + cc], g.two_rho, &trow[cc], &urow[cc]);
  }
}

// -------------------------------------------------------------------------
// Np = 256: a 256x256 complex patch (512 KB) exceeds one CU's LDS, so the
// agent runs as three passes over a chunk of positions, the spectra staged in
// a chunk-sized buffer that is reused every chunk:
//   rows   : a2, a3, forward row DFTs            -> stage
//   cols   : forward column DFTs, a5, inverse column DFTs (in place)
//   rowsinv: inverse row DFTs, a6-a8
// -------------------------------------------------------------------------
constexpr int NP256 = 256;
constexpr int RB = 16;   // rows per workgroup in the row passes
constexpr int CB = 16;   // columns per workgroup in the column pass

__global__ void __launch_bounds__(RB * 16) agent256_rows(AgentArgs g) {
  constexpr int NP = NP256, A = 16, S = NP + A;
  __shared__ float2 tile[RB * S];
  __shared__ float2 tw[NP];
  const int tid = threadIdx.x;
  fill_twiddles<NP>(tw, tid, RB * A);
  const int jl = blockIdx.x / (NP / RB), rb = blockIdx.x % (NP / RB);
  const int j = g.j0 + jl;
  const int2 pj = g.pos[j];
  const int rl = tid / A, p = tid % A, r = rb * RB + rl;
  const float2* xrow = g.xbar + (size_t)(pj.x + r) * g.n2 + pj.y;
  const float2* trow = g.t + (size_t)j * NP * NP + (size_t)r * NP;
  float2 x[16];
#pragma unroll
  for (int nb = 0; nb < 16; ++nb) {
    const int c = p + A * nb;
    const float2 tt = trow[c];
    const float2 xb = xrow[c];
    const float2 v = make_float2(fmaf(g.two_rho, xb.x, tt.x), fmaf(g.two_rho, xb.y, tt.y));
    x[nb] = cmul(g.d[r * NP + c], v);
  }
  __syncthreads();
  row_fwd<NP>(x, tile + rl * S, p, tw);
  float2* out = g.stage + ((size_t)jl * NP + r) * NP;
#pragma unroll
  for (int ka = 0; ka < 16; ++ka) out[p + 16 * ka] = x[ka];
}

__global__ void __launch_bounds__(CB * 16) agent256_cols(AgentArgs g) {
  constexpr int NP = NP256, A = 16;
  __shared__ float2 tile[NP * CB];
  __shared__ float2 tw[NP];
  const int tid = threadIdx.x;
  fill_twiddles<NP>(tw, tid, CB * A);
  const int jl = blockIdx.x / (NP / CB), cb = blockIdx.x % (NP / CB);
  const int j = g.j0 + jl;
  const int c = tid % CB, q = tid / CB, col = cb * CB + c;
  float2* sp = g.stage + (size_t)jl * NP * NP + col;
  float2 x[16];
#pragma unroll
  for (int nb = 0; nb < 16; ++nb) x[nb] = sp[(size_t)(q + A * nb) * NP];
  __syncthreads();
  col_fwd<NP>(x, tile, CB, c, q, tw);
  const float* yc = g.ys + (size_t)j * NP * NP + col;
#pragma unroll
  for (int ka = 0; ka < 16; ++ka) {
    const int k = q + 16 * ka;
    x[ka] = fourier_prox(x[ka], yc[(size_t)k * NP], g.a);
  }
  col_inv<NP>(x, tile, CB, c, q, tw);
#pragma unroll
  for (int nb = 0; nb < 16; ++nb) sp[(size_t)(q + A * nb) * NP] = x[nb];
}

__global__ void __launch_bounds__(RB * 16) agent256_rowsinv(AgentArgs g) {
  constexpr int NP = NP256, A = 16, S = NP + A;
  __shared__ float2 tile[RB * S];
  __shared__ float2 tw[NP];
  const int tid = threadIdx.x;
  fill_twiddles<NP>(tw, tid, RB * A);
  const int jl = blockIdx.x / (NP / RB), rb = blockIdx.x % (NP / RB);
  const int j = g.j0 + jl;
  const int2 pj = g.pos[j];
  const int rl = tid / A, p = tid % A, r = rb * RB + rl;
  float2* io = g.stage + ((size_t)jl * NP + r) * NP;
  float2 x[16];
#pragma unroll
  for (int ka = 0; ka < 16; ++ka) x[ka] = io[p + 16 * ka];
  __syncthreads();
  row_inv<NP>(x, tile + rl * S, p, tw);
  const float2* xrow = g.xbar + (size_t)(pj.x + r) * g.n2 + pj.y;
  float2* trow = g.t + (size_t)j * NP * NP + (size_t)r * NP;
#pragma unroll
  for (int nb = 0; nb < 16; ++nb) {
    const int c = p + A * nb;
    const float2 tt = trow[c];
    const float2 xb = xrow[c];
    const float2 v = make_float2(fmaf(g.two_rho, xb.x, tt.x), fmaf(g.two_rho, xb.y, tt.y));
    finish_pixel(x[nb], v, g.pc[r * NP + c], g.two_rho, &trow[c], &io[c]);
  }
}

// Consensus (eq. (11)) without atomics.  Each thread owns one object pixel
// of a GT_R x GT_C tile and adds the weighted reflections of the chunk's
// patches that cover it, walking the tile's position list (built on the host,
// ascending j).  Chunks run in order on the stream, so every pixel sums its
// contributions in ascending j and the result is bitwise reproducible.
// FUSE: a single chunk holds every position, so the sum is complete and a9
// (xbar, xhat) is finished here.
struct GatherArgs {
  const float2* u;
  const int2* pos;
  const int2* tiles;
  const int* list;
  float2* num;
  const float* laminv;
  float2* xbar;
  float2* xhat;
  unsigned* status;
  int tile0, r0, tiles_c, n1, n2, jbase;
  float rho;
};

template <int NP, bool FUSE>
__global__ void __launch_bounds__(GT_R * GT_C) consensus_gather(GatherArgs g) {
  const int tid = threadIdx.x, bt = blockIdx.x;
  const int2 ti = g.tiles[g.tile0 + bt];
  const int R = g.r0 + (bt / g.tiles_c) * GT_R + tid / GT_C;
  const int C = (bt % g.tiles_c) * GT_C + tid % GT_C;
  float ax = 0.f, ay = 0.f;
#pragma unroll 4
  for (int i = 0; i < ti.y; ++i) {
    const int j = g.list[ti.x + i];
    const int2 pj = g.pos[j];
    const unsigned rr = (unsigned)(R - pj.x), cc = (unsigned)(C - pj.y);
    const bool in = rr < (unsigned)NP && cc < (unsigned)NP;
    // lanes outside the patch read its first pixel and discard it
    const float2 u = g.u[((size_t)(j - g.jbase) * NP + (in ? rr : 0u)) * NP + (in ? cc : 0u)];
    ax += in ? u.x : 0.f;
    ay += in ? u.y : 0.f;
  }
  if (R >= g.n1 || C >= g.n2) return;
  const size_t px = (size_t)R * g.n2 + C;
  if constexpr (FUSE) {
    const float li = g.laminv[px];
    const float2 xb = make_float2(ax * li, ay * li);
    const float2 xh = g.xhat[px];
    g.xbar[px] = xb;
    g.xhat[px] = make_float2(fmaf(g.rho, xb.x - xh.x, xh.x), fmaf(g.rho, xb.y - xh.y, xh.y));
    if (!(isfinite(xb.x) && isfinite(xb.y))) atomicOr(g.status, 1u);
  } else {
    const float2 o = g.num[px];
    g.num[px] = make_float2(o.x + ax, o.y + ay);
  }
}

// -------------------------------------------------------------------------
// a9: consensus image and reconstruction recurrence, accumulator reset.
// -------------------------------------------------------------------------
__global__ void image_update(float2* xbar, float2* xhat, float2* num, const float* laminv, int npx,
                             float rho, unsigned* status) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npx) return;
  const float li = laminv[i];
  const float2 n = num[i];
  const float2 xb = make_float2(n.x * li, n.y * li);
  const float2 xh = xhat[i];
  xbar[i] = xb;
  xhat[i] = make_float2(fmaf(rho, xb.x - xh.x, xh.x), fmaf(rho, xb.y - xh.y, xh.y));
  num[i] = make_float2(0.f, 0.f);
  if (!(isfinite(xb.x) && isfinite(xb.y))) atomicOr(status, 1u);
}

// xhat = Lambda^{-1} num, num <- 0 (reconstruction from a set state)
__global__ void image_from_num(float2* xhat, float2* num, const float* laminv, int npx) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npx) return;
  const float li = laminv[i];
  const float2 n = num[i];
  xhat[i] = make_float2(n.x * li, n.y * li);
  num[i] = make_float2(0.f, 0.f);
}

// -------------------------------------------------------------------------
// init / state kernels
// -------------------------------------------------------------------------
__global__ void init_amplitudes_k(const float* z, float* ys, int np, long long total, float scale,
                                  int centered, unsigned* status) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  long long src = i;
  if (centered) {
    const long long per = (long long)np * np;
    const long long j = i / per;
    const int rem = (int)(i - j * per);
    const int k = rem / np, l = rem - k * np;
    const int h = np / 2;
    src = j * per + (long long)((k + h) % np) * np + (l + h) % np;
  }
  const float zz = z[src];
  if (!(zz >= 0.f) || isinf(zz)) atomicOr(status, 2u);
  ys[i] = scale * sqrtf(fmaxf(zz, 0.f));
}

__global__ void init_patches_k(float2* t, const float2* x0, const int2* pos, int np, int n2,
                               long long total) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const long long per = (long long)np * np;
  const int j = (int)(i / per);
  const int rem = (int)(i - (long long)j * per);
  const int r = rem / np, c = rem - r * np;
  const int2 pj = pos[j];
  t[i] = x0 ? x0[(size_t)(pj.x + r) * n2 + pj.y + c] : make_float2(1.f, 0.f);
}

__global__ void init_images_k(float2* xbar, float2* xhat, float2* num, const float* laminv,
                              const float2* x0, int npx) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npx) return;
  const float2 x = x0 ? x0[i] : make_float2(1.f, 0.f);
  xhat[i] = laminv[i] > 0.f ? x : make_float2(0.f, 0.f);
  xbar[i] = make_float2(0.f, 0.f);
  num[i] = make_float2(0.f, 0.f);
}

__global__ void get_state_k(const float2* t, const float2* xbar, const int2* pos, float2* v, int np,
                            int n2, float two_rho, long long total) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  const long long per = (long long)np * np;
  const int j = (int)(i / per);
  const int rem = (int)(i - (long long)j * per);
  const int r = rem / np, c = rem - r * np;
  const int2 pj = pos[j];
  const float2 xb = xbar[(size_t)(pj.x + r) * n2 + pj.y + c];
  const float2 tt = t[i];
  v[i] = make_float2(fmaf(two_rho, xb.x, tt.x), fmaf(two_rho, xb.y, tt.y));
}

// t <- v and u <- |d|^kappa v for positions [j0, j0 + cnt) (u indexed from j0)
__global__ void set_state_k(float2* t, const float2* v, const float4* pc, float2* u, int np,
                            int j0, long long cnt_px) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt_px) return;
  const long long per = (long long)np * np;
  const long long gi = (long long)j0 * per + i;
  const float2 vv = v[gi];
  t[gi] = vv;
  const float om = pc[i % per].z;
  u[i] = make_float2(om * vv.x, om * vv.y);
}

__global__ void zero_c64_k(float2* a, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = make_float2(0.f, 0.f);
}

// -------------------------------------------------------------------------
// Standalone orthonormal 2-D DFT (operator F of Sec. II and its adjoint).
// -------------------------------------------------------------------------
template <int NP, bool INV>
__global__ void __launch_bounds__(NP * Geo<NP>::A) fft2_small(const float2* in, float2* out) {
  constexpr int A = Geo<NP>::A, B = Geo<NP>::B, S = NP + A, NT = NP * A, M = B / A;
  __shared__ float2 tile[NP * S];
  __shared__ float2 tw[NP];
  const int tid = threadIdx.x;
  fill_twiddles<NP>(tw, tid, NT);
  const size_t base = (size_t)blockIdx.x * NP * NP;
  const float scale = 1.f / NP;
  const int r = tid / A, p = tid % A, c = tid % NP, q = tid / NP;
  float2* row = tile + r * S;
  float2 x[B];
  if constexpr (!INV) {
#pragma unroll
    for (int nb = 0; nb < B; ++nb) x[nb] = in[base + (size_t)r * NP + p + A * nb];
    __syncthreads();
    row_fwd<NP>(x, row, p, tw);
    __syncthreads();
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
      for (int ka = 0; ka < A; ++ka) row[p + A * m + B * ka] = x[m * A + ka];
    __syncthreads();
#pragma unroll
    for (int nb = 0; nb < B; ++nb) x[nb] = tile[(q + A * nb) * S + c];
    col_fwd<NP>(x, tile, S, c, q, tw);
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
      for (int ka = 0; ka < A; ++ka)
        out[base + (size_t)(q + A * m + B * ka) * NP + c] = cscale(x[m * A + ka], scale);
  } else {
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
      for (int ka = 0; ka < A; ++ka) x[m * A + ka] = in[base + (size_t)(q + A * m + B * ka) * NP + c];
    __syncthreads();
    col_inv<NP>(x, tile, S, c, q, tw);
    __syncthreads();
#pragma unroll
    for (int nb = 0; nb < B; ++nb) tile[(q + A * nb) * S + c] = x[nb];
    __syncthreads();
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
      for (int ka = 0; ka < A; ++ka) x[m * A + ka] = row[p + A * m + B * ka];
    row_inv<NP>(x, row, p, tw);
#pragma unroll
    for (int nb = 0; nb < B; ++nb) out[base + (size_t)r * NP + p + A * nb] = cscale(x[nb], scale);
  }
}

// Np = 256 standalone transform: a row pass and a column pass over global memory.
template <bool INV>
__global__ void __launch_bounds__(RB * 16) fft256_rows(const float2* in, float2* out, float scale) {
  constexpr int NP = NP256, A = 16, S = NP + A;
  __shared__ float2 tile[RB * S];
  __shared__ float2 tw[NP];
  const int tid = threadIdx.x;
  fill_twiddles<NP>(tw, tid, RB * A);
  const int jl = blockIdx.x / (NP / RB), rb = blockIdx.x % (NP / RB);
  const int rl = tid / A, p = tid % A, r = rb * RB + rl;
  const size_t base = ((size_t)jl * NP + r) * NP;
  float2 x[16];
  if constexpr (!INV) {
#pragma unroll
    for (int nb = 0; nb < 16; ++nb) x[nb] = in[base + p + A * nb];
    __syncthreads();
    row_fwd<NP>(x, tile + rl * S, p, tw);
#pragma unroll
    for (int ka = 0; ka < 16; ++ka) out[base + p + 16 * ka] = cscale(x[ka], scale);
  } else {
#pragma unroll
    for (int ka = 0; ka < 16; ++ka) x[ka] = in[base + p + 16 * ka];
    __syncthreads();
    row_inv<NP>(x, tile + rl * S, p, tw);
#pragma unroll
    for (int nb = 0; nb < 16; ++nb) out[base + p + A * nb] = cscale(x[nb], scale);
  }
}

template <bool INV>
__global__ void __launch_bounds__(CB * 16) fft256_cols(const float2* in, float2* out, float scale) {
  constexpr int NP = NP256, A = 16;
  __shared__ float2 tile[NP * CB];
  __shared__ float2 tw[NP];
  const int tid = threadIdx.x;
  fill_twiddles<NP>(tw, tid, CB * A);
  const int jl = blockIdx.x / (NP / CB), cb = blockIdx.x % (NP / CB);
  const int c = tid % CB, q = tid / CB, col = cb * CB + c;
  const size_t base = (size_t)jl * NP * NP + col;
  float2 x[16];
  if constexpr (!INV) {
#pragma unroll
    for (int nb = 0; nb < 16; ++nb) x[nb] = in[base + (size_t)(q + A * nb) * NP];
    __syncthreads();
    col_fwd<NP>(x, tile, CB, c, q, tw);
#pragma unroll
    for (int ka = 0; ka < 16; ++ka) out[base + (size_t)(q + 16 * ka) * NP] = cscale(x[ka], scale);
  } else {
#pragma unroll
    for (int ka = 0; ka < 16; ++ka) x[ka] = in[base + (size_t)(q + 16 * ka) * NP];
    __syncthreads();
    col_inv<NP>(x, tile, CB, c, q, tw);
#pragma unroll
    for (int nb = 0; nb < 16; ++nb) out[base + (size_t)(q + A * nb) * NP] = cscale(x[nb], scale);
  }
}

// -------------------------------------------------------------------------
// launchers
// -------------------------------------------------------------------------
static AgentArgs agent_args(const DevState& s, int j0) {
  AgentArgs g;
  g.t = s.t;
  g.ys = s.ys;
  g.pos = s.pos;
  g.d = s.d;
  g.pc = s.pc;
  g.xbar = s.xbar;
  g.num = s.num;
  g.stage = s.stage;
  g.n2 = s.n2;
  g.a = s.a;
  g.two_rho = 2.f * s.rho;
  g.j0 = j0;
  return g;
}

static inline unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

static GatherArgs gather_args(const DevState& s, int g, int jbase) {
  GatherArgs a;
  const int4 ci = s.chunk_info[g];
  a.u = s.stage;
  a.pos = s.pos;
  a.tiles = s.tiles;
  a.list = s.tile_list;
  a.num = reinterpret_cast<float2*>(s.num);
  a.laminv = s.laminv;
  a.xbar = s.xbar;
  a.xhat = s.xhat;
  a.status = s.status;
  a.tile0 = ci.x;
  a.r0 = ci.z;
  a.tiles_c = ci.w;
  a.n1 = s.n1;
  a.n2 = s.n2;
  a.jbase = jbase;
  a.rho = s.rho;
  return a;
}

template <int NP, bool FUSE>
static void gather(const DevState& s, int g, int jbase, hipStream_t st) {
  const int ntiles = s.chunk_info[g].y;
  if (ntiles > 0)
    hipLaunchKernelGGL((consensus_gather<NP, FUSE>), dim3(ntiles), dim3(GT_R * GT_C), 0, st,
                       gather_args(s, g, jbase));
}

hipError_t launch_agent(const DevState& s, hipStream_t st) {
  const AgentArgs g = agent_args(s, 0);
  switch (s.np) {
#define PMACE_AGENT_SMALL(N)                                                        \
  case N:                                                                           \
    hipLaunchKernelGGL(agent_fused<N>, dim3(s.J), dim3(N * Geo<N>::A), 0, st, g);   \
    gather<N, true>(s, 0, 0, st);                                                   \
    break;
    PMACE_AGENT_SMALL(32)
    PMACE_AGENT_SMALL(64)
    PMACE_AGENT_SMALL(128)
#undef PMACE_AGENT_SMALL
    case 256: {
      for (int j0 = 0, gi = 0; j0 < s.J; j0 += s.chunk, ++gi) {
        const int cnt = (s.J - j0 < s.chunk) ? (s.J - j0) : s.chunk;
        const AgentArgs gc = agent_args(s, j0);
        hipLaunchKernelGGL(agent256_rows, dim3(cnt * (NP256 / RB)), dim3(RB * 16), 0, st, gc);
        hipLaunchKernelGGL(agent256_cols, dim3(cnt * (NP256 / CB)), dim3(CB * 16), 0, st, gc);
        hipLaunchKernelGGL(agent256_rowsinv, dim3(cnt * (NP256 / RB)), dim3(RB * 16), 0, st, gc);
        gather<256, false>(s, gi, j0, st);
      }
      const int npx = s.n1 * s.n2;
      hipLaunchKernelGGL(image_update, dim3(blocks_for(npx, 256)), dim3(256), 0, st, s.xbar, s.xhat,
                         reinterpret_cast<float2*>(s.num), s.laminv, npx, s.rho, s.status);
      break;
    }
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_init_amplitudes(const DevState& s, const float* z, float scale, int centered,
                                  hipStream_t st) {
  const long long total = (long long)s.J * s.np * s.np;
  hipLaunchKernelGGL(init_amplitudes_k, dim3(blocks_for(total, 256)), dim3(256), 0, st, z, s.ys, s.np,
                     total, scale, centered, s.status);
  return hipGetLastError();
}

hipError_t launch_init_state(const DevState& s, const float2* x0, hipStream_t st) {
  const long long total = (long long)s.J * s.np * s.np;
  hipLaunchKernelGGL(init_patches_k, dim3(blocks_for(total, 256)), dim3(256), 0, st, s.t, x0, s.pos,
                     s.np, s.n2, total);
  const int npx = s.n1 * s.n2;
  hipLaunchKernelGGL(init_images_k, dim3(blocks_for(npx, 256)), dim3(256), 0, st, s.xbar, s.xhat,
                     reinterpret_cast<float2*>(s.num), s.laminv, x0, npx);
  return hipGetLastError();
}

hipError_t launch_get_state(const DevState& s, float2* v, hipStream_t st) {
  const long long total = (long long)s.J * s.np * s.np;
  hipLaunchKernelGGL(get_state_k, dim3(blocks_for(total, 256)), dim3(256), 0, st, s.t, s.xbar, s.pos,
                     v, s.np, s.n2, 2.f * s.rho, total);
  return hipGetLastError();
}

hipError_t launch_set_state(const DevState& s, const float2* v, hipStream_t st) {
  const int npx = s.n1 * s.n2;
  const long long per = (long long)s.np * s.np;
  hipLaunchKernelGGL(zero_c64_k, dim3(blocks_for(npx, 256)), dim3(256), 0, st,
                     reinterpret_cast<float2*>(s.num), npx);
  hipLaunchKernelGGL(zero_c64_k, dim3(blocks_for(npx, 256)), dim3(256), 0, st, s.xbar, npx);
  for (int j0 = 0, gi = 0; j0 < s.J; j0 += s.chunk, ++gi) {
    const int cnt = (s.J - j0 < s.chunk) ? (s.J - j0) : s.chunk;
    hipLaunchKernelGGL(set_state_k, dim3(blocks_for(cnt * per, 256)), dim3(256), 0, st, s.t, v, s.pc,
                       s.stage, s.np, j0, cnt * per);
    switch (s.np) {
      case 32: gather<32, false>(s, gi, j0, st); break;
      case 64: gather<64, false>(s, gi, j0, st); break;
      case 128: gather<128, false>(s, gi, j0, st); break;
      default: gather<256, false>(s, gi, j0, st); break;
    }
  }
  hipLaunchKernelGGL(image_from_num, dim3(blocks_for(npx, 256)), dim3(256), 0, st, s.xhat,
                     reinterpret_cast<float2*>(s.num), s.laminv, npx);
  return hipGetLastError();
}

hipError_t launch_fft2(int np, int count, const float2* in, float2* out, int inverse, hipStream_t st) {
  switch (np) {
#define PMACE_FFT_SMALL(N)                                                                          \
  case N:                                                                                           \
    if (inverse)                                                                                    \
      hipLaunchKernelGGL((fft2_small<N, true>), dim3(count), dim3(N * Geo<N>::A), 0, st, in, out);  \
    else                                                                                            \
      hipLaunchKernelGGL((fft2_small<N, false>), dim3(count), dim3(N * Geo<N>::A), 0, st, in, out); \
    break;
    PMACE_FFT_SMALL(32)
    PMACE_FFT_SMALL(64)
    PMACE_FFT_SMALL(128)
#undef PMACE_FFT_SMALL
    case 256: {
      const float sc = 1.f / 16.f;  // sqrt(1/256) per pass
      if (inverse) {
        hipLaunchKernelGGL(fft256_cols<true>, dim3(count * (NP256 / CB)), dim3(CB * 16), 0, st, in, out, sc);
        hipLaunchKernelGGL(fft256_rows<true>, dim3(count * (NP256 / RB)), dim3(RB * 16), 0, st, out, out, sc);
      } else {
        hipLaunchKernelGGL(fft256_rows<false>, dim3(count * (NP256 / RB)), dim3(RB * 16), 0, st, in, out, sc);
        hipLaunchKernelGGL(fft256_cols<false>, dim3(count * (NP256 / CB)), dim3(CB * 16), 0, st, out, out, sc);
      }
      break;
    }
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace pmace
