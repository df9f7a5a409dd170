// PMACE iteration kernels for gfx950 (MI355X).
//
// One iteration of Alg. 1 is carried as
//     v_j   = t_j + 2 rho P_j xbar                      (finishes the previous pass's Mann update)
//     w_j   = F_j(v_j)                                  (the data agent, eq. (9))
//     u_j   = 2 w_j - v_j                               (the reflection)
//     t_j  <- v_j - 2 rho w_j                           (first half of the Mann update)
//     xbar  = Lambda^{-1} sum_j P_j^t |d|^kappa u_j     (eq. (11))
//     xhat <- (1 - rho) xhat + rho xbar
// Storing t instead of v is exact algebra of the Mann update (v_new = t + 2 rho P_j xbar),
// and the xhat recurrence is exact algebra of the returned weighted average
// (the average of P_j xbar is xbar on covered pixels; the average of w is the
// mean of the averages of u and v).
//
// The agent applies eq. (9) in the Fourier domain: with W = F(d v),
//     F(d w) = W (alpha + y/|W|) / (1 + alpha)   (0 where W = 0)
// which is the r* of eq. (8) with the phase of W, so w = d^{-1} F^*(...) needs
// one forward and one inverse 2-D DFT per patch.  Where d = 0, eq. (6) leaves
// v free and the agent returns its input there.
//
// PMACE never materialises u.  With U = F(d w) and W = F(d v), the new state
// is t = d^{-1} F^*(W - 2 rho U) (where d != 0), one inverse transform of the
// "state spectrum" W - 2 rho U.  Each state is stored probe-weighted, s = d t
// (t itself where d = 0): the inverse transform is then the new stored state
// as it is, and the next forward frame is d v = s + 2 rho d P_j xbar, so no
// division by d (and no rounding it would amplify) happens in the loop; d^{-1}
// is applied only when a state is read out.  Since u = ((1 - rho) v - t_new) / rho
// and v = t_old + 2 rho P_j xbar, the consensus of eq. (11) is
//     xbar' = 2 (1 - rho) xbar + Lambda^{-1} ((1 - rho) S_old - S_new) / rho,
//     S = sum_j P_j^t |d|^kappa t_j = sum_j P_j^t (|d|^kappa / d) s_j,
// so the gather sums the weighted states themselves and keeps S of the last
// iteration.  Per patch pixel an iteration then reads s and y and writes s
// once, and the consensus reads s once more.
//
// Every kernel reads its reconstruction from a device descriptor (Recon) and
// returns at once when that reconstruction's stop flag is set, so many
// reconstructions can share one launch (work items name the reconstruction).
#include "pmace_dft.hpp"
#include "pmace_internal.hpp"

namespace pmace {

// kRowSpec / kSharpRowSpec: PMACE / SHARP+ on the Np > 128 passes with
// every state kept as the row spectrum of the stored state (see
// agent_rows_body).
constexpr int kPMACE = 0, kSharpPlus = 1, kRowSpec = 2, kSharpRowSpec = 3;
template <int METHOD> constexpr bool row_spec() { return METHOD == kRowSpec || METHOD == kSharpRowSpec; }
template <int METHOD> constexpr bool sharp() { return METHOD == kSharpPlus || METHOD == kSharpRowSpec; }

// Fourier-domain prox of eq. (9): U = W * (a + ys / |W|), 0 where W == 0.
__device__ __forceinline__ float2 fourier_prox(float2 W, float ysv, float a) {
  const float m2 = fmaf(W.x, W.x, W.y * W.y);
  const float rs = m2 > 0.f ? __builtin_amdgcn_rsqf(m2) : 0.f;
  const float g = fmaf(ysv, rs, a);
  return make_float2(W.x * g, W.y * g);
}

// PMACE state spectrum W - 2 rho U = W (tb - 2 rho ys / |W|), tb = 1 - 2 rho a
// (0 where W == 0), scaled by 1/Np^2 (sb = tb/Np^2, s2r = 2 rho/Np^2) so that
// its unnormalised inverse transform is the new stored state d t.
__device__ __forceinline__ float2 state_spectrum(float2 W, float ysv, float sb, float s2r) {
  const float m2 = fmaf(W.x, W.x, W.y * W.y);
  const float rs = m2 > 0.f ? __builtin_amdgcn_rsqf(m2) : 0.f;
  const float g = fmaf(-s2r, ysv * rs, sb);
  return make_float2(W.x * g, W.y * g);
}

// Where the agent works on the spectrum: PMACE forms the state spectrum,
// SHARP+ the magnitude projection (a = 0).
template <int METHOD>
__device__ __forceinline__ float2 spectrum_step(float2 W, float ysv, const Recon& g) {
  if constexpr (!sharp<METHOD>()) return state_spectrum(W, ysv, g.sb, g.s2r);
  else return fourier_prox(W, ysv, 0.f);
}

__device__ __forceinline__ float2 mann_v(float2 t, float2 xb, float two_rho) {
  return make_float2(fmaf(two_rho, xb.x, t.x), fmaf(two_rho, xb.y, t.y));
}

// Prologue (a2-a3): the frame that is transformed.
//   PMACE : d v = s + 2 rho d P_j xbar       (v of Alg. 1 times the probe, from the
//                                             stored s = d t; 0 where d == 0)
//   SHARP+: t + 2 beta d P_j xbar            (the frame s of Alg. 2)
template <int METHOD>
__device__ __forceinline__ float2 agent_input(float2 s, float2 xb, float2 d, float two_rho) {
  const float2 dx = cmul(d, xb);
  if constexpr (METHOD == kPMACE) {
    const bool nz = d.x != 0.f || d.y != 0.f;
    return make_float2(fmaf(two_rho, dx.x, nz ? s.x : 0.f), fmaf(two_rho, dx.y, nz ? s.y : 0.f));
  } else {
    return mann_v(s, dx, two_rho);
  }
}

// Epilogue (a6-a8) from the unnormalised inverse transform z of the spectrum
// step's output, for probe pixel k.
//   PMACE : z = F^*((W - 2 rho U)/Np^2) is the new d t, stored as it is.  Where
//           d == 0 the agent returns its input, w = v, so the state there is
//           t <- (1 - 2 rho) v (the old state and xbar are read only at such
//           pixels, and only for a probe with zeros).  No u is written.
//   SHARP+: a = z/Np^2 = P_a s; the next state t = (1 - 2 beta) a + beta s -
//           beta d P_j xbar (P_Q s of this iteration is d P_j xbar of the last
//           one: P_Q is a projection, so P_Q s_{k+1} = P_Q P_a s_k), and the
//           overlap numerator takes conj(d) a.  pc = {conj(d)/Np^2, conj(d)}.
// SHARP+ epilogue with the old state t_old = *tp already loaded.
__device__ __forceinline__ void sharp_output(float2 z, float2 t_old, float2* tp, const float2* xp, int k,
                                             const Recon& g, float2* u_out) {
  const float4 pcf = g.pc[k];
  const float2 dx = cmul(make_float2(pcf.z, -pcf.w), *xp);
  const float2 sv = mann_v(t_old, dx, g.two_rho);
  *tp = make_float2(fmaf(g.ka, z.x, g.beta * (sv.x - dx.x)), fmaf(g.ka, z.y, g.beta * (sv.y - dx.y)));
  *u_out = cmul(make_float2(pcf.x, pcf.y), z);
}
template <int METHOD>
__device__ __forceinline__ void agent_output(float2 z, float2* tp, const float2* xp, int k,
                                             const Recon& g, float2* u_out) {
  if constexpr (METHOD == kPMACE) {
    float2 sn = z;
    if (g.has_zero) {
      const float2 dk = g.d[k];
      if (dk.x == 0.f && dk.y == 0.f) sn = cscale(mann_v(*tp, *xp, g.two_rho), 1.f - g.two_rho);
    }
    *tp = sn;
  } else {
    sharp_output(z, *tp, tp, xp, k, g, u_out);
  }
}

// -------------------------------------------------------------------------
// Np <= 128: the whole patch lives in LDS; one workgroup per work item
// (reconstruction, position) does a2-a7 in one pass (rows, columns, state
// spectrum, columns, rows, new state).
// -------------------------------------------------------------------------
__device__ __forceinline__ float2 cfma(float2 a, float2 b, float2 acc) {
  return make_float2(fmaf(a.x, b.x, fmaf(-a.y, b.y, acc.x)), fmaf(a.x, b.y, fmaf(a.y, b.x, acc.y)));
}
// acc - a * b
__device__ __forceinline__ float2 cfms(float2 a, float2 b, float2 acc) {
  return make_float2(fmaf(-a.x, b.x, fmaf(a.y, b.y, acc.x)), fmaf(-a.x, b.y, fmaf(-a.y, b.x, acc.y)));
}

// PPW patches per workgroup: sub-group threadIdx.x / NT works on patch j with
// its own tile; the twiddle table is shared.  A sub-group with live == false
// (past the last position, or a stopped batch member) runs every step and
// barrier on a valid patch j but stores nothing.
template <int NP, int METHOD, int PPW = 1>
__device__ __forceinline__ void agent_fused_body(const Recon& g, const int j, const bool live = true) {
  constexpr int A = Geo<NP>::A, B = Geo<NP>::B, S = NP + A, NT = NP * A, M = B / A;
  static_assert(exch_phases<NP>() == 1, "the whole-patch tile exchanges in one round");
  static_assert(PPW * NT <= 1024, "patches per workgroup: at most 1024 threads");
  __shared__ float2 tile_all[PPW * NP * S];
  __shared__ float2 tw[NP];
  const int sub = PPW > 1 ? (int)threadIdx.x / NT : 0;
  const int tid = PPW > 1 ? (int)threadIdx.x - sub * NT : (int)threadIdx.x;
  float2* tile = tile_all + sub * (NP * S);
  const int2 pj = g.pos[j];
  const size_t pb = (size_t)j * NP * NP;
  const int r = tid / A, p = tid % A;
  const float2* xrow = g.xbar + (size_t)(pj.x + r) * g.n2 + pj.y;
  float2* trow = g.t + pb + (size_t)r * NP;
  const float two_rho = g.two_rho;

  float2 x[B];
#pragma unroll
  for (int nb = 0; nb < B; ++nb) {
    const int c = p + A * nb;
    x[nb] = agent_input<METHOD>(trow[c], xrow[c], g.d[r * NP + c], two_rho);
  }
  // the twiddle table after the frame's loads, so the two are in flight
  // together (the row transforms wait for both anyway)
  if (sub == 0) load_twiddles<NP>(tw, g.twn, tid, NT);
  // amplitudes of the column phase, fetched now so their latency hides
  // behind the row transforms
  const int c = tid % NP, q = tid / NP;
  const float* yc = g.ys + pb + c;
  float yv[B];
#pragma unroll
  for (int m = 0; m < M; ++m)
#pragma unroll
    for (int ka = 0; ka < A; ++ka) yv[m * A + ka] = yc[(size_t)(q + A * m + B * ka) * NP];
  __syncthreads();
  float2* row = tile + r * S;
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
    for (int ka = 0; ka < A; ++ka) x[m * A + ka] = spectrum_step<METHOD>(x[m * A + ka], yv[m * A + ka], g);
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
  if (!live) return;   // no barrier follows

  float2* urow = g.stage + pb + (size_t)r * NP;  // SHARP+ only
#pragma unroll
  for (int nb = 0; nb < B; ++nb) {
    const int cc = p + A * nb;
    agent_output<METHOD>(x[nb], &trow[cc], &xrow[cc], r * NP + cc, g, &urow[cc]);
  }
}

// One reconstruction (descriptor passed by value): block b handles positions
// b PPW ... b PPW + PPW - 1.
template <int NP, int METHOD, int PPW>
__global__ void __launch_bounds__(PPW * NP * Geo<NP>::A) agent_fused(const Recon g) {
  constexpr int NT = NP * Geo<NP>::A;
  if constexpr (PPW == 1) {
    agent_fused_body<NP, METHOD>(g, blockIdx.x);
  } else {
    const int j = (int)blockIdx.x * PPW + (int)threadIdx.x / NT;
    const bool live = j < g.J;
    agent_fused_body<NP, METHOD, PPW>(g, live ? j : g.J - 1, live);
  }
}

// Batched: block b handles work items (reconstruction, position) b PPW ...
// b PPW + PPW - 1 of the nitems; a block all of whose items belong to stopped
// members returns at once (the test is the same in every thread).
template <int NP, int PPW>
__global__ void __launch_bounds__(PPW * NP * Geo<NP>::A) agent_fused_batch(
    const Recon* __restrict__ recs, const int2* __restrict__ items, int nitems) {
  constexpr int NT = NP * Geo<NP>::A;
  if constexpr (PPW == 1) {
    const int2 it = items[blockIdx.x];
    const Recon& g = recs[it.x];
    if (*g.done) return;
    agent_fused_body<NP, kPMACE>(g, it.y);
  } else {
    const int i0 = (int)blockIdx.x * PPW;
    bool any = false;
    for (int s = 0; s < PPW && i0 + s < nitems; ++s) any |= *recs[items[i0 + s].x].done == 0;
    if (!any) return;
    const int i = i0 + (int)threadIdx.x / NT;
    const int2 it = items[i < nitems ? i : nitems - 1];
    const Recon& g = recs[it.x];
    agent_fused_body<NP, kPMACE, PPW>(g, it.y, i < nitems && *g.done == 0);
  }
}

// The window term of two coset blocks, (a, 0) and (a, 1), of position j at
// once: each product (2 rho d) xbar is loaded once and added to both blocks
// with the signs (-1)^{a q1 + b q2}, so a workgroup doing both blocks reads
// the probe and the consensus window half as often per block.  Block (a, b)
// at (rr, c) is
//   Z_ab[rr][c] + W_Np^{a rr + b c} sum_q (-1)^{a q1 + b q2} (2 rho d)[(rr, c) + M q] xbar[p_j + (rr, c) + M q].
// The quadrant loop is kept rolled, so one quadrant's loads are in flight at a
// time (they are L2 hits: the probe table and the consensus image); the state
// blocks, read from HBM, are loaded last.  twnp: W_Np^m, m < Np, in LDS.
template <int M, int NB0, int NB1>
__device__ __forceinline__ void split_frame_pair(const Recon& g, const int j, const int a, const int rr,
                                                 const int p, const float2* twnp, float2 (&x0)[Geo<M>::B],
                                                 float2 (&x1)[Geo<M>::B]) {
  constexpr int A = Geo<M>::A, NP = 2 * M, NB = NB1 - NB0;
  const int2 pj = g.pos[j];
#pragma unroll
  for (int nb = NB0; nb < NB1; ++nb) x0[nb] = x1[nb] = make_float2(0.f, 0.f);
#pragma unroll 1
  for (int q = 0; q < 4; ++q) {
    const int q1 = q >> 1, q2 = q & 1;
    const float2* dq = g.dr + (size_t)(rr + M * q1) * NP + M * q2;
    const float2* xq = g.xbar + (size_t)(pj.x + rr + M * q1) * g.n2 + pj.y + M * q2;
    float2 dv[NB], xv[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
      dv[k] = dq[p + A * (NB0 + k)];
      xv[k] = xq[p + A * (NB0 + k)];
    }
    if ((a * q1) & 1) {            // block (a, 0); uniform across the workgroup
#pragma unroll
      for (int k = 0; k < NB; ++k) x0[NB0 + k] = cfms(dv[k], xv[k], x0[NB0 + k]);
    } else {
#pragma unroll
      for (int k = 0; k < NB; ++k) x0[NB0 + k] = cfma(dv[k], xv[k], x0[NB0 + k]);
    }
    if ((a * q1 + q2) & 1) {       // block (a, 1)
#pragma unroll
      for (int k = 0; k < NB; ++k) x1[NB0 + k] = cfms(dv[k], xv[k], x1[NB0 + k]);
    } else {
#pragma unroll
      for (int k = 0; k < NB; ++k) x1[NB0 + k] = cfma(dv[k], xv[k], x1[NB0 + k]);
    }
  }
  int ri = rr;
  asm volatile("" : "+v"(ri));
  const float2* z0 = g.t + ((size_t)j * 4 + 2 * a) * M * M + (size_t)ri * M;
  const float2* z1 = z0 + (size_t)M * M;
#pragma unroll
  for (int nb = NB0; nb < NB1; ++nb) {
    const int c = p + A * nb;
    x0[nb] = cfma(twnp[a * ri], x0[nb], z0[c]);
    x1[nb] = cfma(twnp[a * ri + c], x1[nb], z1[c]);
  }
#pragma unroll
  for (int nb = NB0; nb < NB1; ++nb) {
    asm volatile("" : "+v"(x0[nb].x), "+v"(x0[nb].y));
    asm volatile("" : "+v"(x1[nb].x), "+v"(x1[nb].y));
  }
}

// One split block from its frame x (row layout) to its new state: the M x M
// DFT of the block is the patch spectrum at the frequencies (2 k1 + a,
// 2 k2 + b); the state spectrum is formed there with the amplitudes stored
// in the same order, and 4 x its unnormalised inverse is the block of the new
// state (the inverse of the split step gives 4 s' per block).  The M-point
// transforms use W_M^m = W_Np^{2m}.
template <int M>
__device__ __forceinline__ void split_block_pass(const Recon& g, const size_t pb, float2 (&x)[Geo<M>::B],
                                                 float2* tile, const float2* tw) {
  constexpr int A = Geo<M>::A, B = Geo<M>::B, S = M + A, MB = B / A;
  const int tid = threadIdx.x;
  const int r = tid / A, p = tid % A, c = tid % M, q = tid / M;
  const float* yc = g.ys + pb + c;
  float yv[B];
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int ka = 0; ka < A; ++ka) yv[m * A + ka] = yc[(size_t)(q + A * m + B * ka) * M];
  __syncthreads();
  float2* row = tile + r * S;
  row_fwd<M>(x, row, p, tw);
  __syncthreads();
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int ka = 0; ka < A; ++ka) row[p + A * m + B * ka] = x[m * A + ka];
  __syncthreads();
#pragma unroll
  for (int nb = 0; nb < B; ++nb) x[nb] = tile[(q + A * nb) * S + c];
  col_fwd<M>(x, tile, S, c, q, tw);
  {
    const float sb = 4.f * g.sb, s2r = 4.f * g.s2r;   // exact: powers of two
#pragma unroll
    for (int k = 0; k < B; ++k) x[k] = state_spectrum(x[k], yv[k], sb, s2r);
  }
  col_inv<M>(x, tile, S, c, q, tw);
  __syncthreads();
#pragma unroll
  for (int nb = 0; nb < B; ++nb) tile[(q + A * nb) * S + c] = x[nb];
  __syncthreads();
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int ka = 0; ka < A; ++ka) x[m * A + ka] = row[p + A * m + B * ka];
  row_inv<M>(x, row, p, tw);
  float2* z = g.t + pb + (size_t)r * M;
#pragma unroll
  for (int nb = 0; nb < B; ++nb) z[p + A * nb] = x[nb];
}

// Split layout, two coset blocks per workgroup: blocks (a, 0) and (a, 1) of
// one position share their window loads (split_frame_pair), then run one
// after the other through the block transforms.
template <int M>
__device__ __forceinline__ void agent_split_pair_body(const Recon& g, const int j, const int a) {
  constexpr int A = Geo<M>::A, B = Geo<M>::B, S = M + A, NT = M * A;
  __shared__ float2 tile[M * S];
  __shared__ float2 tw[M];
  __shared__ float2 twnp[2 * M];
  const int tid = threadIdx.x;
  for (int m = tid; m < 2 * M; m += NT) twnp[m] = g.twn[m];
  __syncthreads();
  for (int m = tid; m < M; m += NT) tw[m] = twnp[2 * m];
  const int r = tid / A, p = tid % A;
  float2 x0[B], x1[B];
  split_frame_pair<M, 0, B / 2>(g, j, a, r, p, twnp, x0, x1);
  split_frame_pair<M, B / 2, B>(g, j, a, r, p, twnp, x0, x1);
  split_block_pass<M>(g, ((size_t)j * 4 + 2 * a) * M * M, x0, tile, tw);
  split_block_pass<M>(g, ((size_t)j * 4 + 2 * a + 1) * M * M, x1, tile, tw);
}

// Block b: position xcd * jper + (b / 8) / 2, row of cosets a = (b / 8) mod 2
// (the two workgroups of a position on one XCD, back to back).
template <int M>
__global__ void __launch_bounds__(M * Geo<M>::A) agent_split_pair(const Recon g, int check_done, int jper) {
  if (check_done && *g.done) return;
  const int b = blockIdx.x, slot = b >> 3;
  const int j = (b & 7) * jper + (slot >> 1);
  if (j >= g.J) return;
  agent_split_pair_body<M>(g, j, slot & 1);
}


// -------------------------------------------------------------------------
// Np in {160, 192, 256}: the patch (up to 512 KB) exceeds one CU's LDS, so
// the agent runs as three passes over a chunk of positions, the spectra
// staged in a chunk-sized buffer that is reused every chunk:
//   rows   : a2, a3, forward row DFTs            -> stage
//   cols   : forward column DFTs, spectrum step (a5), inverse column DFTs (in place)
//   rowsinv: inverse row DFTs, a6-a7 (t); SHARP+: stage <- overlap numerators
// A workgroup takes rb_of<NP>() rows (row passes) or CB columns (column pass) of one
// patch, with Geo<NP>::A threads per line.
// -------------------------------------------------------------------------
constexpr int RB = PMACE_RB;        // rows per workgroup in the row passes (160, 192)
constexpr int RB256 = PMACE_RB256;  // ... and for 256-point lines (tuned apart)
constexpr int CB = PMACE_CB;   // columns per workgroup in the column pass
static_assert(RB >= 4 && RB <= 32 && 160 % RB == 0 && 192 % RB == 0, "row block");
static_assert(RB256 >= 4 && RB256 <= 32 && 256 % RB256 == 0, "row block (256)");
template <int NP> constexpr int rb_of() { return NP == 256 ? RB256 : RB; }
static_assert(CB >= 8 && CB <= 32 && 160 % CB == 0 && 192 % CB == 0 && 256 % CB == 0, "column block");
template <int NP> constexpr int row_threads() { return rb_of<NP>() * Geo<NP>::A; }
template <int NP> constexpr int col_threads() { return CB * Geo<NP>::A; }

// A store that does not keep its line in the caches (data read back only
// after far more than the caches hold has passed through them).
typedef float pm_f2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void store_nt(float2* p, float2 v) {
  const pm_f2v t = {v.x, v.y};
  __builtin_nontemporal_store(t, reinterpret_cast<pm_f2v*>(p));
}

template <int NP, int METHOD, bool NT>
__device__ __forceinline__ void agent_rows_body(const Recon& g, const int j0) {
  constexpr int A = Geo<NP>::A, B = Geo<NP>::B, M = B / A, S = row_cap<NP>();
  constexpr int RBn = rb_of<NP>();
  __shared__ float2 tile[RBn * S];
  __shared__ float2 tw[NP];
  const int tid = threadIdx.x;
  // PMACE: the table is written to LDS once the loads below are issued;
  // SHARP+ loads it first (each measured the faster for its method)
  TwiddleFetch<NP, RBn * A> twf;
  if constexpr (METHOD != kSharpPlus) twf.fetch(g.twn, tid);
  else load_twiddles<NP>(tw, g.twn, tid, RBn * A);
  const int jl = blockIdx.x / (NP / RBn), rb = blockIdx.x % (NP / RBn);
  const int j = j0 + jl;
  const int2 pj = g.pos[j];
  const int rl = tid / A, p = tid % A, r = rb * RBn + rl;
  const float2* xrow = g.xbar + (size_t)(pj.x + r) * g.n2 + pj.y;
  const float2* trow = g.t + (size_t)j * NP * NP + (size_t)r * NP;
  float2 x[B];
  if constexpr (row_spec<METHOD>()) {
    // The state is kept as H = F_r(s)/Np (its row spectrum, natural order),
    // so the frame's row spectrum is Np H + F_r(2 rho d P_j xbar): only the
    // window term is transformed here (SHARP+: 2 beta for 2 rho, and t for s).  H is fetched first, in the order the
    // transform leaves its output, so its latency hides behind the transform.
    float2 h[B];
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
      for (int ka = 0; ka < A; ++ka) h[m * A + ka] = trow[p + A * m + B * ka];
#pragma unroll
    for (int nb = 0; nb < B; ++nb) {
      const int c = p + A * nb;
      x[nb] = cscale(cmul(g.d[r * NP + c], xrow[c]), g.two_rho);
    }
    twf.store(tw, tid);
    __syncthreads();
    row_fwd<NP>(x, tile + rl * S, p, tw);
    constexpr float fnp = (float)NP;
#pragma unroll
    for (int k = 0; k < B; ++k) x[k] = make_float2(fmaf(fnp, h[k].x, x[k].x), fmaf(fnp, h[k].y, x[k].y));
  } else {
#pragma unroll
    for (int nb = 0; nb < B; ++nb) {
      const int c = p + A * nb;
      x[nb] = agent_input<METHOD>(trow[c], xrow[c], g.d[r * NP + c], g.two_rho);
    }
    if constexpr (METHOD == kPMACE) twf.store(tw, tid);
    __syncthreads();
    row_fwd<NP>(x, tile + rl * S, p, tw);
  }
  float2* out = g.stage + ((size_t)jl * NP + r) * NP;
#pragma unroll
  for (int m = 0; m < M; ++m)
#pragma unroll
    for (int ka = 0; ka < A; ++ka) {
      if constexpr (NT) store_nt(out + p + A * m + B * ka, x[m * A + ka]);
      else out[p + A * m + B * ka] = x[m * A + ka];
    }
}

// NT: the stage (and, in the column pass, the new row-spectrum states) written
// past the caches, for stages far larger than the Infinity Cache
template <int NP, int METHOD, bool NT = false>
__global__ void __launch_bounds__(row_threads<NP>()) agent_rows(const Recon g, int j0) {
  agent_rows_body<NP, METHOD, NT>(g, j0);
}

// Batch members: the member's descriptor by value (global, not flat, loads),
// its stop flag read through it.
template <int NP, int METHOD, bool NT = false>
__global__ void __launch_bounds__(row_threads<NP>()) agent_rows_batch(const Recon g, int j0) {
  if (*g.done) return;
  agent_rows_body<NP, METHOD, NT>(g, j0);
}

template <int NP, int METHOD, bool NT>
__device__ __forceinline__ void agent_cols_body(const Recon& g, const int j0) {
  constexpr int A = Geo<NP>::A, B = Geo<NP>::B, M = B / A;
  __shared__ float2 tile[col_rows<NP>() * CB];
  __shared__ float2 tw[NP];
  const int tid = threadIdx.x;
  // PMACE: the table is written to LDS once the loads below are issued;
  // SHARP+ loads it first (each measured the faster for its method)
  TwiddleFetch<NP, CB * A> twf;
  if constexpr (METHOD != kSharpPlus) twf.fetch(g.twn, tid);
  else load_twiddles<NP>(tw, g.twn, tid, CB * A);
  const int jl = blockIdx.x / (NP / CB), cb = blockIdx.x % (NP / CB);
  const int j = j0 + jl;
  const int c = tid % CB, q = tid / CB, col = cb * CB + c;
  float2* sp = g.stage + (size_t)jl * NP * NP + col;
  float2 x[B];
#pragma unroll
  for (int nb = 0; nb < B; ++nb) x[nb] = sp[(size_t)(q + A * nb) * NP];
  // SHARP+ on row-spectrum states: the part of the next state that does not
  // depend on the projection, ((2 beta - 1)/(2 Np)) F_r(s) + T/2, formed from
  // this pass's input and the old state now (both loads hide behind the
  // transforms), so the input need not be read again at the end
  float2 ysr[METHOD == kSharpRowSpec ? B : 1];
  if constexpr (METHOD == kSharpRowSpec) {
    const float2* tp = g.t + (size_t)j * NP * NP + col;
    const float c1 = (g.two_rho - 1.f) / (2.f * (float)NP);
#pragma unroll
    for (int nb = 0; nb < B; ++nb) {
      const float2 to = tp[(size_t)(q + A * nb) * NP];
      ysr[nb] = make_float2(fmaf(c1, x[nb].x, 0.5f * to.x), fmaf(c1, x[nb].y, 0.5f * to.y));
    }
  }
  // amplitudes of the spectrum step, fetched now so their latency hides
  // behind the forward column transforms
  const float* yc = g.ys + (size_t)j * NP * NP + col;
  float yv[B];
#pragma unroll
  for (int m = 0; m < M; ++m)
#pragma unroll
    for (int ka = 0; ka < A; ++ka) yv[m * A + ka] = yc[(size_t)(q + A * m + B * ka) * NP];
  if constexpr (METHOD != kSharpPlus) twf.store(tw, tid);
  __syncthreads();
  col_fwd<NP>(x, tile, CB, c, q, tw);
#pragma unroll
  for (int k = 0; k < B; ++k) x[k] = spectrum_step<METHOD>(x[k], yv[k], g);
  col_inv<NP>(x, tile, CB, c, q, tw);
  if constexpr (METHOD == kSharpRowSpec) {
    // SHARP+ with row-spectrum states T = F_r(t)/Np: the column inverse C of
    // the magnitude projection gives P_a s = F_r^*(C)/Np^2, and the next state
    // t' = (1 - 2 beta) P_a s + beta (s - d P_j xbar) with s = t + 2 beta d P_j xbar
    // is, in row spectra, T' = ka C + ((2 beta - 1)/(2 Np)) F_r(s) + T/2, where
    // F_r(s) is this pass's input (the last two terms are ysr, formed above).
    // C goes back to the stage for the overlap projection (through the
    // caches: the consensus reads it next; with NT the new state does not).
    float2* tp = g.t + (size_t)j * NP * NP + col;
#pragma unroll
    for (int nb = 0; nb < B; ++nb) {
      const size_t o = (size_t)(q + A * nb) * NP;
      const float2 tn = make_float2(fmaf(g.ka, x[nb].x, ysr[nb].x), fmaf(g.ka, x[nb].y, ysr[nb].y));
      if constexpr (NT) store_nt(tp + o, tn);
      else tp[o] = tn;
      sp[o] = x[nb];
    }
  } else {
    // kRowSpec: the column inverse of the state spectrum is F_r(s_new)/Np, the
    // new state itself; the inverse row pass is left to the consensus
    float2* op = METHOD == kRowSpec ? g.t + (size_t)j * NP * NP + col : sp;
#pragma unroll
    for (int nb = 0; nb < B; ++nb) {
      if constexpr (NT && METHOD == kRowSpec) store_nt(op + (size_t)(q + A * nb) * NP, x[nb]);
      else op[(size_t)(q + A * nb) * NP] = x[nb];
    }
  }
}

template <int NP, int METHOD, bool NT = false>
__global__ void __launch_bounds__(col_threads<NP>()) agent_cols(const Recon g, int j0) {
  agent_cols_body<NP, METHOD, NT>(g, j0);
}

template <int NP, int METHOD, bool NT = false>
__global__ void __launch_bounds__(col_threads<NP>()) agent_cols_batch(const Recon g, int j0) {
  if (*g.done) return;
  agent_cols_body<NP, METHOD, NT>(g, j0);
}

template <int NP, int METHOD>
__device__ __forceinline__ void agent_rowsinv_body(const Recon& g, const int j0) {
  constexpr int A = Geo<NP>::A, B = Geo<NP>::B, M = B / A, S = row_cap<NP>();
  constexpr int RBn = rb_of<NP>();
  __shared__ float2 tile[RBn * S];
  __shared__ float2 tw[NP];
  const int tid = threadIdx.x;
  // PMACE: the table is written to LDS once the loads below are issued;
  // SHARP+ loads it first (each measured the faster for its method)
  TwiddleFetch<NP, RBn * A> twf;
  if constexpr (METHOD == kPMACE) twf.fetch(g.twn, tid);
  else load_twiddles<NP>(tw, g.twn, tid, RBn * A);
  const int jl = blockIdx.x / (NP / RBn), rb = blockIdx.x % (NP / RBn);
  const int j = j0 + jl;
  const int2 pj = g.pos[j];
  const int rl = tid / A, p = tid % A, r = rb * RBn + rl;
  float2* io = g.stage + ((size_t)jl * NP + r) * NP;
  const float2* xrow = g.xbar + (size_t)(pj.x + r) * g.n2 + pj.y;
  float2* trow = g.t + (size_t)j * NP * NP + (size_t)r * NP;
  float2 x[B];
#pragma unroll
  for (int m = 0; m < M; ++m)
#pragma unroll
    for (int ka = 0; ka < A; ++ka) x[m * A + ka] = io[p + A * m + B * ka];
  // SHARP+ needs the old state again: fetched now, behind the transform
  // (not for 40-point lines, where the registers would halve occupancy)
  constexpr bool kOldAhead = METHOD == kSharpPlus && B <= 24;
  float2 t_old[B];
  if constexpr (kOldAhead) {
#pragma unroll
    for (int nb = 0; nb < B; ++nb) t_old[nb] = trow[p + A * nb];
  }
  if constexpr (METHOD == kPMACE) twf.store(tw, tid);
  __syncthreads();
  row_inv<NP>(x, tile + rl * S, p, tw);
#pragma unroll
  for (int nb = 0; nb < B; ++nb) {
    const int c = p + A * nb;
    if constexpr (kOldAhead) sharp_output(x[nb], t_old[nb], &trow[c], &xrow[c], r * NP + c, g, &io[c]);
    else agent_output<METHOD>(x[nb], &trow[c], &xrow[c], r * NP + c, g, &io[c]);
  }
}

template <int NP, int METHOD>
__global__ void __launch_bounds__(row_threads<NP>()) agent_rowsinv(const Recon g, int j0) {
  agent_rowsinv_body<NP, METHOD>(g, j0);
}

template <int NP>
__global__ void __launch_bounds__(row_threads<NP>()) agent_rowsinv_batch(const Recon g, int j0) {
  if (*g.done) return;
  agent_rowsinv_body<NP, kPMACE>(g, j0);
}

// -------------------------------------------------------------------------
// Consensus (eq. (11)) without atomics.  Each thread owns one object pixel
// of a GT_R x GT_C tile and adds the contributions of the patches that cover
// it, walking the tile's position list (built on the host, ascending j):
//   PMACE : |d|^kappa t_j = (|d|^kappa / d) s_j, |d|^kappa t_j where d == 0 (the
//           sum S of the weighted states),
//   SHARP+: the overlap numerators conj(d) P_a s_j left in the stage buffer
//           (`jbase` = first position held there).
// Np > 128 chunks run in order on the stream, so every pixel sums its
// contributions in ascending j and the result is bitwise reproducible.  FUSE
// (Np <= 128, every position in one chunk): the sum is complete, so a9 (xbar,
// xhat) is finished here; otherwise it is added to num.
// -------------------------------------------------------------------------

// The per-pixel images the a9 update reads, loaded ahead of the sum that
// it combines them with.
struct ImageIn {
  float li;
  float2 so, xo, xh;
};
template <int METHOD>
__device__ __forceinline__ ImageIn load_image_in(const Recon& g, size_t px) {
  ImageIn v;
  v.li = g.laminv[px];
  if constexpr (METHOD == kPMACE) {
    v.so = g.sold[px];
    v.xo = g.xbar[px];
  }
  v.xh = g.xhat[px];
  return v;
}
// a9 for one object pixel from the complete sum S.
template <int METHOD>
__device__ __forceinline__ void finish_image(const Recon& g, size_t px, float2 S, const ImageIn& v) {
  float2 xb;
  if constexpr (METHOD == kPMACE) {
    const float ex = fmaf(g.co, v.so.x, -g.cn * S.x), ey = fmaf(g.co, v.so.y, -g.cn * S.y);
    xb = make_float2(fmaf(g.cx, v.xo.x, v.li * ex), fmaf(g.cx, v.xo.y, v.li * ey));
    g.sold[px] = S;
  } else {
    xb = make_float2(S.x * v.li, S.y * v.li);
  }
  g.xbar[px] = xb;
  g.xhat[px] = make_float2(fmaf(g.rho, xb.x - v.xh.x, v.xh.x), fmaf(g.rho, xb.y - v.xh.y, v.xh.y));
  if (!(isfinite(xb.x) && isfinite(xb.y))) atomicOr(g.status, 1u);
}
template <int METHOD>
__device__ __forceinline__ void finish_image(const Recon& g, size_t px, float2 S) {
  finish_image<METHOD>(g, px, S, load_image_in<METHOD>(g, px));
}

#define PM_STR(x) #x
#define PM_UNROLL(n) _Pragma(PM_STR(unroll n))

template <int NP, bool FUSE, int METHOD>
__device__ __forceinline__ void consensus_gather_body(const Recon& g, const int tile, const int jbase) {
  constexpr int NPX = GT_R * GT_C, NT = GT_THREADS, LIST = 256;
  __shared__ int3 sl[LIST];  // (patch slot, row, col) of the listed positions
  const int tid = threadIdx.x;
  // GT_K threads share a pixel: part k sums list entries k, k + GT_K, ...
  const int pxl = tid % NPX, part = tid / NPX;
  const int4 ti = g.tiles[tile];
  const int R = ti.z + pxl / GT_C, C = ti.w + pxl % GT_C;
  // the pixel's thread (part 0) loads what it combines the sum with now, so
  // those loads overlap the list and state loads instead of following them
  const bool own = part == 0 && R < g.n1 && C < g.n2;
  const size_t px = own ? (size_t)R * g.n2 + C : 0;
  ImageIn img{};
  float2 acc0 = make_float2(0.f, 0.f);
  if (own) {
    if constexpr (FUSE) img = load_image_in<METHOD>(g, px);
    else acc0 = g.num[px];
  }
  const float2* src = METHOD == kPMACE ? g.t : g.stage;
  const int jb = METHOD == kPMACE ? 0 : jbase;
  float ax = 0.f, ay = 0.f;
  for (int b0 = 0; b0 < ti.y; b0 += LIST) {
    const int nb = ti.y - b0 < LIST ? ti.y - b0 : LIST;
    if (b0 > 0) __syncthreads();
    for (int i = tid; i < nb; i += NT) {
      const int j = g.tile_list[ti.x + b0 + i];
      const int2 pj = g.pos[j];
      sl[i] = make_int3(j - jb, pj.x, pj.y);
    }
    __syncthreads();
    PM_UNROLL(PMACE_GATHER_UNROLL)
    for (int i = part; i < nb; i += GT_K) {
      const int3 e = sl[i];
      const unsigned rr = (unsigned)(R - e.y), cc = (unsigned)(C - e.z);
      const bool in = rr < (unsigned)NP && cc < (unsigned)NP;
      // lanes outside the patch read its first pixel and discard it
      const unsigned o = in ? rr * NP + cc : 0u;
      const float2 u = src[(size_t)e.x * NP * NP + o];
      if constexpr (METHOD == kPMACE) {
        const float2 w = in ? g.gw[o] : make_float2(0.f, 0.f);
        ax = fmaf(w.x, u.x, fmaf(-w.y, u.y, ax));
        ay = fmaf(w.x, u.y, fmaf(w.y, u.x, ay));
      } else {
        ax += in ? u.x : 0.f;
        ay += in ? u.y : 0.f;
      }
    }
  }
  if constexpr (GT_K > 1) {
    // partial sums added in a fixed order: still bitwise reproducible
    __shared__ float2 ps[(GT_K > 1 ? GT_K - 1 : 1) * NPX];
    if (part > 0) ps[(part - 1) * NPX + pxl] = make_float2(ax, ay);
    __syncthreads();
    if (part > 0) return;
#pragma unroll
    for (int k = 0; k < GT_K - 1; ++k) {
      ax += ps[k * NPX + pxl].x;
      ay += ps[k * NPX + pxl].y;
    }
  }
  if (!own) return;
  if constexpr (FUSE) {
    finish_image<METHOD>(g, px, make_float2(ax, ay), img);
  } else {
    g.num[px] = make_float2(acc0.x + ax, acc0.y + ay);
  }
}

// One reconstruction: block b handles tile first_tile + b.
template <int NP, bool FUSE, int METHOD>
__global__ void __launch_bounds__(GT_THREADS) consensus_gather(const Recon g, int first_tile,
                                                                int jbase) {
  consensus_gather_body<NP, FUSE, METHOD>(g, first_tile + blockIdx.x, jbase);
}

// One batch member (descriptor in device memory): block b handles tile first_tile + b.
template <int NP, bool FUSE>
__global__ void __launch_bounds__(GT_THREADS) consensus_gather_member(const Recon g, int first_tile,
                                                                       int jbase) {
  if (*g.done) return;
  consensus_gather_body<NP, FUSE, kPMACE>(g, first_tile + blockIdx.x, jbase);
}

// Batched: block b handles work item (reconstruction, tile) b.
template <int NP, bool FUSE>
__global__ void __launch_bounds__(GT_THREADS) consensus_gather_batch(const Recon* __restrict__ recs,
                                                                      const int2* __restrict__ items,
                                                                      int jbase) {
  const int2 it = items[blockIdx.x];
  const Recon& g = recs[it.x];
  if (*g.done) return;
  consensus_gather_body<NP, FUSE, kPMACE>(g, it.y, jbase);
}

// -------------------------------------------------------------------------
// Consensus for states kept as row spectra: PMACE (kRowSpec) sums
// S = sum_j P_j^t (|d|^kappa / d) s_j with s_j = F_r^*(H_j) (the stored
// H_j = F_r(s_j)/Np); SHARP+ (kSharpRowSpec) sums the overlap numerators
// sum_j P_j^t conj(d) P_a s_j with P_a s_j = F_r^*(C_j)/Np^2, C_j left in the
// stage by the column pass (`jbase` = first position held there).  The
// inverse row transforms thus run here instead of in a pass of their own.  A
// row of a patch lands on one object row: a workgroup owns one object row R
// (a CR_W-pixel segment of it) and walks its list of the chunk's positions
// whose patch covers R and meets the segment, with entries (j, row of P_j on
// R, patch column), in rounds of cr_rows<NP>() entries grouped by patch row,
// each round sorted by patch column.  Each round inverse-transforms its patch
// rows in LDS and weights them; every thread then adds, in list order, the
// ones that cover its pixel of R.  Every pixel's sum thus runs in one fixed
// order (chunks in turn, then the list), with no atomics: bitwise
// reproducible.  CHECK: batch member, skip when stopped.  FUSE (every
// position in one chunk): each pixel's sum is complete, so a9 is finished
// here instead of adding the sum to num.
// -------------------------------------------------------------------------
// patch rows per round: CR_T threads' worth, at most 64 (LDS)
template <int NP> constexpr int cr_rows() { return CR_T / Geo<NP>::A < 64 ? CR_T / Geo<NP>::A : 64; }
template <int NP> constexpr int cr_threads() { return cr_rows<NP>() * Geo<NP>::A; }
// (at least NP + 1: a row keeps a zero at index NP for the sums below; where
// the transform's own span is shorter, NP + 4 sets consecutive rows 8 banks
// apart, so the row groups of a wave do not collide in its LDS exchange)
template <int NP> constexpr int cr_pitch() { return row_cap<NP>() > NP ? row_cap<NP>() : NP + 4; }

template <int NP, bool CHECK, int METHOD, bool FUSE>
__global__ void __launch_bounds__(cr_threads<NP>()) consensus_rows(const Recon g, int first_item,
                                                                    int jbase) {
  static_assert(row_spec<METHOD>(), "row-spectrum states");
  if constexpr (CHECK) {
    if (*g.done) return;
  }
  constexpr int A = Geo<NP>::A, B = Geo<NP>::B, M = B / A, S = cr_pitch<NP>(), RN = cr_rows<NP>();
  constexpr int NT = cr_threads<NP>(), PX = CR_W / NT;
  static_assert(CR_W % NT == 0 && NT % 64 == 0, "row segment over the workgroup");
  __shared__ float2 rows[RN * S];
  __shared__ float2 tw[NP];
  __shared__ int pcol[RN];
  const int tid = threadIdx.x, rl = tid / A, p = tid % A;
  const int4 it = g.citems[first_item + blockIdx.x];  // (list start, count, object row, first column)
  TwiddleFetch<NP, NT> twf;
  twf.fetch(g.twn, tid);
  // this row group's entry of a round, its patch row (in the order the
  // inverse transform takes it) and the weights of that row
  int4 en;
  float2 x[B], w[B];
  auto fetch = [&](int e) {
    en = e < it.y ? g.clist[it.x + e] : make_int4(jbase, 0, 0, 0);
    const float2* hr = METHOD == kSharpRowSpec
                           ? g.stage + (size_t)(en.x - jbase) * NP * NP + (size_t)en.y * NP
                           : g.t + (size_t)en.x * NP * NP + (size_t)en.y * NP;
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
      for (int ka = 0; ka < A; ++ka) x[m * A + ka] = hr[p + A * m + B * ka];
#pragma unroll
    for (int nb = 0; nb < B; ++nb) {
      if constexpr (METHOD == kSharpRowSpec) {
        const float4 pcf = g.pc[en.y * NP + p + A * nb];  // {conj(d)/Np^2, conj(d)}
        w[nb] = make_float2(pcf.x, pcf.y);
      } else {
        w[nb] = g.gw[en.y * NP + p + A * nb];
      }
    }
  };
  fetch(rl);
  twf.store(tw, tid);
  float ax[PX], ay[PX];
#pragma unroll
  for (int k = 0; k < PX; ++k) ax[k] = ay[k] = 0.f;
  const int lane0 = __builtin_amdgcn_readfirstlane(tid & ~63);  // first pixel (relative) of this wave
  const int w0 = __builtin_amdgcn_readfirstlane(it.w);
  for (int e0 = 0; e0 < it.y; e0 += RN) {
    const int ne = it.y - e0 < RN ? it.y - e0 : RN;
    __syncthreads();  // the last round's sums are done with rows[]; tw is written
    row_inv<NP>(x, rows + rl * S, p, tw);
    wave_sync();
    if (p == 0) {
      pcol[rl] = en.z;
      rows[rl * S + NP] = make_float2(0.f, 0.f);
    }
#pragma unroll
    for (int nb = 0; nb < B; ++nb) rows[rl * S + p + A * nb] = cmul(w[nb], x[nb]);
    __syncthreads();
    // Lane e of every wave holds entry e's patch column (past the round's
    // entries: above any column).  The list is sorted by patch column, so the
    // entries covering some of a wave's 64 pixels [cw, cw + 64) are the lanes
    // [lo, hi) with cw - NP < pc <= cw + 63, counted by two ballots; each
    // pixel adds the ones that cover it, in list order.  An entry that does
    // not cover the pixel adds the row's zero at index NP instead, so the
    // loop has no branch and keeps several LDS reads in flight.
    const int lane = tid & 63;
    const int pv = lane < ne ? pcol[lane] : 0x7fffffff;
#pragma unroll
    for (int k = 0; k < PX; ++k) {
      const int cw = w0 + lane0 + k * NT;
      const int lo = __popcll(__ballot(pv <= cw - NP));
      const int hi = __popcll(__ballot(pv <= cw + 63));
      const int C = cw + lane;
      auto at = [&](int e) {
        const unsigned cc = (unsigned)(C - __builtin_amdgcn_readlane(pv, e));
        return rows[e * S + (cc < (unsigned)NP ? cc : (unsigned)NP)];
      };
      int e = lo;
      for (; e + 4 <= hi; e += 4) {
        const float2 v0 = at(e), v1 = at(e + 1), v2 = at(e + 2), v3 = at(e + 3);
        ax[k] = ((ax[k] + v0.x) + v1.x + v2.x) + v3.x;
        ay[k] = ((ay[k] + v0.y) + v1.y + v2.y) + v3.y;
      }
      for (; e < hi; ++e) {
        const float2 v = at(e);
        ax[k] += v.x;
        ay[k] += v.y;
      }
    }
    if (e0 + RN < it.y) fetch(e0 + RN + rl);
  }
  const size_t row0 = (size_t)it.z * g.n2;
#pragma unroll
  for (int k = 0; k < PX; ++k) {
    const int C = it.w + tid + k * NT;
    if (C < g.n2) {
      if constexpr (FUSE) {
        finish_image<METHOD == kSharpRowSpec ? kSharpPlus : kPMACE>(g, row0 + C, make_float2(ax[k], ay[k]));
      } else {
        const float2 o = g.num[row0 + C];
        g.num[row0 + C] = make_float2(o.x + ax[k], o.y + ay[k]);
      }
    }
  }
}

// a9 for Np > 128: consensus image, reconstruction recurrence, accumulator reset.
__device__ __forceinline__ void image_update_body(const Recon& g) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n1 * g.n2) return;
  const float2 n = g.num[i];
  if (g.method == kSharpPlus) finish_image<kSharpPlus>(g, i, n);
  else finish_image<kPMACE>(g, i, n);
  g.num[i] = make_float2(0.f, 0.f);
}

__global__ void image_update(const Recon g) { image_update_body(g); }

__global__ void image_update_batch(const Recon g) {
  if (*g.done) return;
  image_update_body(g);
}

// After the states were set from outside (xbar = 0, t = v): xhat = the
// weighted average Lambda^{-1} num of the states; PMACE keeps S = num.
// num <- 0.
__global__ void image_from_num(const Recon* __restrict__ rec) {
  const Recon& g = *rec;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n1 * g.n2) return;
  const float li = g.laminv[i];
  const float2 n = g.num[i];
  g.xhat[i] = make_float2(n.x * li, n.y * li);
  if (g.method == kPMACE) g.sold[i] = n;
  g.num[i] = make_float2(0.f, 0.f);
}

// PMACE after init: S of the initial states; num <- 0.
__global__ void sold_from_num(const Recon* __restrict__ rec) {
  const Recon& g = *rec;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n1 * g.n2) return;
  g.sold[i] = g.num[i];
  g.num[i] = make_float2(0.f, 0.f);
}

// -------------------------------------------------------------------------
// a10: NRMSE (eq. (17)) of xhat against a reference, per reconstruction.
// theta = arg sum conj(xref) xhat minimises the numerator, so
//   e^2 = (sum |xhat|^2 + sum |xref|^2 - 2 |sum conj(xref) xhat|) / sum |xref|^2.
// Two deterministic stages: per-block FP64 partial sums (wavefront shuffles,
// then the waves in order), then one block per reconstruction sums the
// partials the same way.
// -------------------------------------------------------------------------
// Sums v[0..N) over a block of RED_T threads: a butterfly of wavefront
// shuffles inside each wave, then the per-wave sums added in wave order by
// thread 0 (the only thread whose v holds the totals afterwards).  The order
// is fixed, so the result is bitwise reproducible.
template <int N>
__device__ __forceinline__ void block_sum(double (&v)[N]) {
  static_assert(RED_T % 64 == 0 && RED_T <= 1024, "whole wavefronts");
#pragma unroll
  for (int off = 32; off > 0; off >>= 1)
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] += __shfl_xor(v[q], off);
  __shared__ double ws[N][RED_T / 64];
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int q = 0; q < N; ++q) ws[q][w] = v[q];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < N; ++q) {
      double t = ws[q][0];
      for (int k = 1; k < RED_T / 64; ++k) t += ws[q][k];
      v[q] = t;
    }
}

// update_stop = 0 evaluates on demand, also for stopped reconstructions.
__global__ void __launch_bounds__(RED_T) nrmse_partial(const Recon* __restrict__ recs,
                                                       const int2* __restrict__ items, int update_stop) {
  const int2 it = items[blockIdx.x];
  const Recon& g = recs[it.x];
  if ((update_stop && *g.done) || !g.xref) return;
  const int npx = g.n1 * g.n2;
  const int base = it.y * RED_PX;
  // every load of the thread's pixels is issued before the sums (one memory
  // round trip, not one per pixel); the sums then run in the same order
  constexpr int PER = RED_PX / RED_T;
  float2 xr[PER], xh[PER];
  bool on[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    const int i = base + (int)threadIdx.x + u * RED_T;
    const int ic = i < npx ? i : 0;
    on[u] = i < npx && (!g.mask || g.mask[ic]);
    xr[u] = g.xref[ic];
    xh[u] = g.xhat[ic];
  }
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int u = 0; u < PER; ++u) {
    if (on[u]) {
      acc[0] += (double)xr[u].x * xh[u].x + (double)xr[u].y * xh[u].y;   // Re conj(xref) xhat
      acc[1] += (double)xr[u].x * xh[u].y - (double)xr[u].y * xh[u].x;   // Im conj(xref) xhat
      acc[2] += (double)xh[u].x * xh[u].x + (double)xh[u].y * xh[u].y;   // |xhat|^2
      acc[3] += (double)xr[u].x * xr[u].x + (double)xr[u].y * xr[u].y;   // |xref|^2
    }
  }
  block_sum<4>(acc);
  if (threadIdx.x == 0)
    for (int q = 0; q < 4; ++q) g.red[4 * it.y + q] = acc[q];
}

__global__ void __launch_bounds__(RED_T) nrmse_finish(const Recon* __restrict__ recs,
                                                      const int* __restrict__ items, int update_stop,
                                                      float tol, int min_iter) {
  const Recon& g = recs[items[blockIdx.x]];
  if ((update_stop && *g.done) || !g.xref) return;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < g.n_red; b += RED_T)
    for (int q = 0; q < 4; ++q) acc[q] += g.red[4 * b + q];
  block_sum<4>(acc);
  if (threadIdx.x != 0) return;
  const double sref = acc[3];
  const double c = sqrt(acc[0] * acc[0] + acc[1] * acc[1]);
  const double e2 = (acc[2] + sref - 2.0 * c) / (sref > 0.0 ? sref : 1.0);
  const double e = sqrt(e2 > 0.0 ? e2 : 0.0);
  const double prev = g.track[1];
  g.track[0] = sref;
  g.track[2] = prev;
  g.track[1] = e;
  // stop rule: NRMSE change below tol once min_iter iterations have run
  if (update_stop && g.track[3] >= (double)min_iter && fabs(e - prev) < (double)tol) *g.done = 1;
}

// -------------------------------------------------------------------------
// Truth-free stop rule: the data-fit cost of eq. (4) at the current
// reconstruction, C = sum_j f_j(P_j xhat) = 1/2 sum_j ||y_j - |F D P_j xhat|||^2
// (sigma_n = 1; only its relative change is used).  With the unnormalised
// transform W = Np F(D P_j xhat) and yfac * ys = Np y_j, each patch adds
// (yfac ys - |W|)^2 / (2 Np^2).  Per-patch (Np > 128: per column block)
// partial sums in FP64, summed per reconstruction in a fixed order.
// -------------------------------------------------------------------------
__device__ __forceinline__ void block_sum_to(float v, double* out, double scale) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  __shared__ double wsum[16];
  const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) wsum[w] = (double)v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < nw; ++i) s += wsum[i];
    *out = s * scale;
  }
}

__device__ __forceinline__ float fit_term(float2 W, float yv) {
  const float m = sqrtf(fmaf(W.x, W.x, W.y * W.y));
  const float e = yv - m;
  return e * e;
}

template <int NP>
__device__ __forceinline__ void fit_small_body(const Recon& g, const int j) {
  constexpr int A = Geo<NP>::A, B = Geo<NP>::B, S = NP + A, NT = NP * A, M = B / A;
  static_assert(exch_phases<NP>() == 1, "the whole-patch tile exchanges in one round");
  __shared__ float2 tile[NP * S];
  __shared__ float2 tw[NP];
  const int tid = threadIdx.x;
  load_twiddles<NP>(tw, g.twn, tid, NT);
  const int2 pj = g.pos[j];
  const int r = tid / A, p = tid % A;
  const float2* xrow = g.xhat + (size_t)(pj.x + r) * g.n2 + pj.y;
  float2 x[B];
#pragma unroll
  for (int nb = 0; nb < B; ++nb) {
    const int c = p + A * nb;
    x[nb] = cmul(g.d[r * NP + c], xrow[c]);
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
  const float* yc = g.ys + (size_t)j * NP * NP + c;
  float acc = 0.f;
#pragma unroll
  for (int m = 0; m < M; ++m)
#pragma unroll
    for (int ka = 0; ka < A; ++ka)
      acc += fit_term(x[m * A + ka], g.yfac * yc[(size_t)(q + A * m + B * ka) * NP]);
  block_sum_to(acc, &g.fit[j], 0.5 / ((double)NP * NP));
}

template <int NP>
__global__ void __launch_bounds__(NP * Geo<NP>::A) fit_small(const Recon* __restrict__ rec) {
  fit_small_body<NP>(*rec, blockIdx.x);
}

template <int NP>
__global__ void __launch_bounds__(NP * Geo<NP>::A) fit_small_batch(const Recon* __restrict__ recs,
                                                                   const int2* __restrict__ items) {
  const int2 it = items[blockIdx.x];
  const Recon& g = recs[it.x];
  if (*g.done) return;
  fit_small_body<NP>(g, it.y);
}

// Np > 128: rows pass of F(D P_j xhat) into the stage, then columns + cost.
template <int NP>
__global__ void __launch_bounds__(row_threads<NP>()) fit_rows(const Recon* __restrict__ rec, int j0,
                                                               int check_done) {
  const Recon& g = *rec;
  if (check_done && *g.done) return;
  constexpr int A = Geo<NP>::A, B = Geo<NP>::B, M = B / A, S = row_cap<NP>();
  constexpr int RBn = rb_of<NP>();
  __shared__ float2 tile[RBn * S];
  __shared__ float2 tw[NP];
  const int tid = threadIdx.x;
  TwiddleFetch<NP, RBn * A> twf;  // written to LDS once the loads below are issued
  twf.fetch(g.twn, tid);
  const int jl = blockIdx.x / (NP / RBn), rb = blockIdx.x % (NP / RBn);
  const int2 pj = g.pos[j0 + jl];
  const int rl = tid / A, p = tid % A, r = rb * RBn + rl;
  const float2* xrow = g.xhat + (size_t)(pj.x + r) * g.n2 + pj.y;
  float2 x[B];
#pragma unroll
  for (int nb = 0; nb < B; ++nb) {
    const int c = p + A * nb;
    x[nb] = cmul(g.d[r * NP + c], xrow[c]);
  }
  twf.store(tw, tid);
  __syncthreads();
  row_fwd<NP>(x, tile + rl * S, p, tw);
  float2* out = g.stage + ((size_t)jl * NP + r) * NP;
#pragma unroll
  for (int m = 0; m < M; ++m)
#pragma unroll
    for (int ka = 0; ka < A; ++ka) out[p + A * m + B * ka] = x[m * A + ka];
}

template <int NP>
__global__ void __launch_bounds__(col_threads<NP>()) fit_cols(const Recon* __restrict__ rec, int j0,
                                                               int check_done) {
  const Recon& g = *rec;
  if (check_done && *g.done) return;
  constexpr int A = Geo<NP>::A, B = Geo<NP>::B, M = B / A;
  __shared__ float2 tile[col_rows<NP>() * CB];
  __shared__ float2 tw[NP];
  const int tid = threadIdx.x;
  TwiddleFetch<NP, CB * A> twf;  // written to LDS once the loads below are issued
  twf.fetch(g.twn, tid);
  const int jl = blockIdx.x / (NP / CB), cb = blockIdx.x % (NP / CB);
  const int j = j0 + jl;
  const int c = tid % CB, q = tid / CB, col = cb * CB + c;
  const float2* sp = g.stage + (size_t)jl * NP * NP + col;
  float2 x[B];
#pragma unroll
  for (int nb = 0; nb < B; ++nb) x[nb] = sp[(size_t)(q + A * nb) * NP];
  // amplitudes fetched now, behind the column transforms
  const float* yc = g.ys + (size_t)j * NP * NP + col;
  float yv[B];
#pragma unroll
  for (int m = 0; m < M; ++m)
#pragma unroll
    for (int ka = 0; ka < A; ++ka) yv[m * A + ka] = yc[(size_t)(q + A * m + B * ka) * NP];
  twf.store(tw, tid);
  __syncthreads();
  col_fwd<NP>(x, tile, CB, c, q, tw);
  float acc = 0.f;
#pragma unroll
  for (int k = 0; k < B; ++k) acc += fit_term(x[k], g.yfac * yv[k]);
  block_sum_to(acc, &g.fit[(size_t)j * (NP / CB) + cb], 0.5 / ((double)NP * NP));
}

// Sum the partials per reconstruction; the truth-free rule stops a member when
// |C_k - C_{k-1}| <= tol C_{k-1} once min_iter iterations have run.
__global__ void __launch_bounds__(RED_T) fit_finish(const Recon* __restrict__ recs,
                                                    const int* __restrict__ items, int update_stop,
                                                    float tol, int min_iter) {
  const Recon& g = recs[items[blockIdx.x]];
  if (update_stop && *g.done) return;
  const int n = g.J * g.fit_bpp;
  double acc[1] = {0.0};
  for (int i = threadIdx.x; i < n; i += RED_T) acc[0] += g.fit[i];
  block_sum<1>(acc);
  if (threadIdx.x != 0) return;
  const double cst = acc[0];
  if (!update_stop) {  // on demand: leaves the stop rule's history alone
    g.track[6] = cst;
    return;
  }
  const double prev = g.track[4];
  g.track[5] = prev;
  g.track[4] = cst;
  if (g.track[3] >= (double)min_iter && isfinite(prev) && fabs(cst - prev) <= (double)tol * prev)
    *g.done = 1;
}

// One iteration done: count it for every member that ran it (before the
// stop rule is evaluated), or (cap) stop members that reached max_iter.
__global__ void tick_k(const Recon* __restrict__ recs, const int* __restrict__ items, int n,
                       int max_iter, int cap) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const Recon& g = recs[items[i]];
  if (*g.done) return;
  if (cap) {
    if (g.track[3] >= (double)max_iter) *g.done = 1;
  } else {
    g.track[3] += 1.0;
  }
}

// -------------------------------------------------------------------------
// init / state kernels
// -------------------------------------------------------------------------
__global__ void init_amplitudes_k(const Recon* __restrict__ rec, const float* z, float scale,
                                  int centered) {
  const Recon& g = *rec;
  const long long per = (long long)g.np * g.np;
  const long long total = per * g.J;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= total) return;
  long long src = i;
  if (centered || g.split) {
    const long long j = i / per;
    const int rem = (int)(i - j * per);
    int k = rem / g.np, l = rem - k * g.np;
    if (g.split) {  // element m of coset block ab holds the frequency (2 m1 + a, 2 m2 + b)
      const int M = g.np / 2, ab = rem / (M * M), m = rem - ab * M * M;
      k = 2 * (m / M) + (ab >> 1);
      l = 2 * (m % M) + (ab & 1);
    }
    const int h = centered ? g.np / 2 : 0;
    src = j * per + (long long)((k + h) % g.np) * g.np + (l + h) % g.np;
  }
  const float zz = z[src];
  if (!(zz >= 0.f) || isinf(zz)) atomicOr(g.status, 2u);
  g.ys[i] = scale * sqrtf(fmaxf(zz, 0.f));
}

__global__ void init_patches_k(const Recon* __restrict__ rec, const float2* x0) {
  const Recon& g = *rec;
  const long long per = (long long)g.np * g.np;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= per * g.J) return;
  const int j = (int)(i / per);
  const int rem = (int)(i - (long long)j * per);
  const int r = rem / g.np, c = rem - r * g.np;
  const int2 pj = g.pos[j];
  const float2 x = x0 ? x0[(size_t)(pj.x + r) * g.n2 + pj.y + c] : make_float2(1.f, 0.f);
  // Alg. 1: v_j = P_j x0 (= t, xbar = 0), stored as d t (t where d == 0).
  // Alg. 2: s_j = D P_j x0, held as t = s - 2 beta d P_j xbar with xbar = x0
  // (the overlap image of consistent frames), i.e. (1 - 2 beta) d x0.
  const float2 dd = g.d[rem];
  if (g.method == kSharpPlus) g.t[i] = cscale(cmul(dd, x), 1.f - g.two_rho);
  else g.t[i] = (dd.x != 0.f || dd.y != 0.f) ? cmul(dd, x) : x;
}

// Lambda = sum_j P_j^t omega (eq. (11)) in FP64 over one chunk's tiles, each
// pixel adding its covering positions in ascending j (chunks run in order),
// into `lam` (the accumulator image viewed as FP64, zeroed first).
__global__ void __launch_bounds__(GT_THREADS) lambda_gather_k(const Recon* __restrict__ rec,
                                                             int first_tile, double* __restrict__ lam) {
  const Recon& g = *rec;
  const int4 ti = g.tiles[first_tile + blockIdx.x];
  const int np = g.np;
  for (int px = threadIdx.x; px < GT_R * GT_C; px += blockDim.x) {
    const int R = ti.z + px / GT_C, C = ti.w + px % GT_C;
    if (R >= g.n1 || C >= g.n2) continue;
    double acc = 0.0;
    for (int i = 0; i < ti.y; ++i) {
      const int2 pj = g.pos[g.tile_list[ti.x + i]];
      const unsigned rr = (unsigned)(R - pj.x), cc = (unsigned)(C - pj.y);
      if (rr < (unsigned)np && cc < (unsigned)np) acc += g.omega64[rr * np + cc];
    }
    lam[(size_t)R * g.n2 + C] += acc;
  }
}

// Lambda^{-1}, 0 where Lambda = 0 (no patch, or only zero weights, covers the pixel).
__global__ void laminv_k(const Recon* __restrict__ rec, const double* __restrict__ lam) {
  const Recon& g = *rec;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n1 * g.n2) return;
  g.laminv[i] = lam[i] != 0.0 ? (float)(1.0 / lam[i]) : 0.f;
}

__global__ void zero_f64_k(double* __restrict__ a, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) a[i] = 0.0;
}

__global__ void init_images_k(const Recon* __restrict__ rec, const float2* x0) {
  const Recon& g = *rec;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n1 * g.n2) return;
  const float2 x = x0 ? x0[i] : make_float2(1.f, 0.f);
  g.xhat[i] = g.laminv[i] > 0.f ? x : make_float2(0.f, 0.f);
  g.xbar[i] = g.method == kSharpPlus ? g.xhat[i] : make_float2(0.f, 0.f);
  g.num[i] = make_float2(0.f, 0.f);
}

// src: the probe-weighted states (t itself, or their row-spectrum form
// already transformed back into v, which is then rewritten in place).
__global__ void get_state_k(const Recon* __restrict__ rec, const float2* src, float2* v) {
  const Recon& g = *rec;
  const long long per = (long long)g.np * g.np;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= per * g.J) return;
  const int j = (int)(i / per);
  const int rem = (int)(i - (long long)j * per);
  const int r = rem / g.np, c = rem - r * g.np;
  const int2 pj = g.pos[j];
  const float2 xb = g.xbar[(size_t)(pj.x + r) * g.n2 + pj.y + c];
  // PMACE: v = t + 2 rho P_j xbar with t = d^{-1} s (dinv = d^{-1}/Np^2; s where
  // d == 0);  SHARP+: s = t + 2 beta d P_j xbar
  if (g.method == kSharpPlus) {
    v[i] = mann_v(src[i], cmul(g.d[rem], xb), g.two_rho);
  } else {
    const float2 di = g.dinv[rem], s = src[i];
    const float2 t = (di.x != 0.f || di.y != 0.f) ? cscale(cmul(di, s), g.np2f) : s;
    v[i] = mann_v(t, xb, g.two_rho);
  }
}

// t <- v for positions [j0, j0 + cnt), PMACE stored as d v (v where d == 0);
// SHARP+ also stage <- conj(d) v (the weights of eq. (15), stage indexed from
// j0).  PMACE's gather weights the stored states themselves.
__global__ void set_state_k(const Recon* __restrict__ rec, const float2* v, int j0, long long cnt_px) {
  const Recon& g = *rec;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= cnt_px) return;
  const long long per = (long long)g.np * g.np;
  const long long gi = (long long)j0 * per + i;
  const float2 vv = v[gi];
  if (g.method == kSharpPlus) {
    g.t[gi] = vv;
    const float4 pcf = g.pc[i % per];
    g.stage[i] = cmul(make_float2(pcf.z, pcf.w), vv);
  } else {
    const float2 dd = g.d[i % per];
    g.t[gi] = (dd.x != 0.f || dd.y != 0.f) ? cmul(dd, vv) : vv;
  }
}

// SHARP+ after set_state: xbar = the overlap image of s (just left in xhat),
// then t = s - 2 beta d P_j xbar so that s = t + 2 beta d P_j xbar.
__global__ void sharp_image_k(const Recon* __restrict__ rec) {
  const Recon& g = *rec;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n1 * g.n2) return;
  g.xbar[i] = g.xhat[i];
}

__global__ void sharp_state_k(const Recon* __restrict__ rec) {
  const Recon& g = *rec;
  const long long per = (long long)g.np * g.np;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= per * g.J) return;
  const int j = (int)(i / per);
  const int rem = (int)(i - (long long)j * per);
  const int r = rem / g.np, c = rem - r * g.np;
  const int2 pj = g.pos[j];
  const float2 dx = cmul(g.d[rem], g.xbar[(size_t)(pj.x + r) * g.n2 + pj.y + c]);
  const float2 t = g.t[i];
  g.t[i] = make_float2(fmaf(-g.two_rho, dx.x, t.x), fmaf(-g.two_rho, dx.y, t.y));
}

__global__ void zero_images_k(const Recon* __restrict__ rec) {
  const Recon& g = *rec;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n1 * g.n2) return;
  g.num[i] = make_float2(0.f, 0.f);
  g.xbar[i] = make_float2(0.f, 0.f);
}

// -------------------------------------------------------------------------
// Standalone orthonormal 2-D DFT (operator F of Sec. II and its adjoint).
// -------------------------------------------------------------------------
template <int NP, bool INV>
__global__ void __launch_bounds__(NP * Geo<NP>::A) fft2_small(const float2* in, float2* out) {
  constexpr int A = Geo<NP>::A, B = Geo<NP>::B, S = NP + A, NT = NP * A, M = B / A;
  static_assert(exch_phases<NP>() == 1, "the whole-patch tile exchanges in one round");
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

// Np > 128 standalone transform: a row pass and a column pass over global memory.
template <int NP, bool INV>
__global__ void __launch_bounds__(row_threads<NP>()) fft_rows(const float2* in, float2* out, float scale) {
  constexpr int A = Geo<NP>::A, B = Geo<NP>::B, M = B / A, S = row_cap<NP>();
  constexpr int RBn = rb_of<NP>();
  __shared__ float2 tile[RBn * S];
  __shared__ float2 tw[NP];
  const int tid = threadIdx.x;
  fill_twiddles<NP>(tw, tid, RBn * A);
  const int jl = blockIdx.x / (NP / RBn), rb = blockIdx.x % (NP / RBn);
  const int rl = tid / A, p = tid % A, r = rb * RBn + rl;
  const size_t base = ((size_t)jl * NP + r) * NP;
  float2 x[B];
  if constexpr (!INV) {
#pragma unroll
    for (int nb = 0; nb < B; ++nb) x[nb] = in[base + p + A * nb];
    __syncthreads();
    row_fwd<NP>(x, tile + rl * S, p, tw);
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
      for (int ka = 0; ka < A; ++ka) out[base + p + A * m + B * ka] = cscale(x[m * A + ka], scale);
  } else {
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
      for (int ka = 0; ka < A; ++ka) x[m * A + ka] = in[base + p + A * m + B * ka];
    __syncthreads();
    row_inv<NP>(x, tile + rl * S, p, tw);
#pragma unroll
    for (int nb = 0; nb < B; ++nb) out[base + p + A * nb] = cscale(x[nb], scale);
  }
}

template <int NP, bool INV>
__global__ void __launch_bounds__(col_threads<NP>()) fft_cols(const float2* in, float2* out, float scale) {
  constexpr int A = Geo<NP>::A, B = Geo<NP>::B, M = B / A;
  __shared__ float2 tile[col_rows<NP>() * CB];
  __shared__ float2 tw[NP];
  const int tid = threadIdx.x;
  fill_twiddles<NP>(tw, tid, CB * A);
  const int jl = blockIdx.x / (NP / CB), cb = blockIdx.x % (NP / CB);
  const int c = tid % CB, q = tid / CB, col = cb * CB + c;
  const size_t base = (size_t)jl * NP * NP + col;
  float2 x[B];
  if constexpr (!INV) {
#pragma unroll
    for (int nb = 0; nb < B; ++nb) x[nb] = in[base + (size_t)(q + A * nb) * NP];
    __syncthreads();
    col_fwd<NP>(x, tile, CB, c, q, tw);
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
      for (int ka = 0; ka < A; ++ka)
        out[base + (size_t)(q + A * m + B * ka) * NP] = cscale(x[m * A + ka], scale);
  } else {
#pragma unroll
    for (int m = 0; m < M; ++m)
#pragma unroll
      for (int ka = 0; ka < A; ++ka) x[m * A + ka] = in[base + (size_t)(q + A * m + B * ka) * NP];
    __syncthreads();
    col_inv<NP>(x, tile, CB, c, q, tw);
#pragma unroll
    for (int nb = 0; nb < B; ++nb) out[base + (size_t)(q + A * nb) * NP] = cscale(x[nb], scale);
  }
}

// -------------------------------------------------------------------------
// Split layout (Np = 2M): consensus, image update, states, data fit
// -------------------------------------------------------------------------
// Consensus sum S = sum_j P_j^t (|d|^kappa / d) s_j from split-layout states.
// A workgroup owns a QT_R x QT_C base tile T; for every position whose
// quadrant-0 block [p_j, p_j + M)^2 meets T (list ascending in j), each pixel
// of T at m = R - p_j undoes the split step from the four blocks at m,
//     s[m + M q] = 1/4 sum_ab (-1)^{a q1 + b q2} W_Np^{-(a m1 + b m2)} Z_ab[m],
// and adds the weighted values to the pixels T + M q: one partial sum per
// quadrant q, written to part[q] (each block value is read once).  QT_K
// threads share a pixel, thread k taking the entries k, k + QT_K, ...; their
// sums are added in the order k = 0..QT_K-1.  The image update adds the four
// partials in the order q = 0..3.
template <int M>
__device__ __forceinline__ void consensus_split_body(const Recon& g, const int tile) {
  constexpr int NP = 2 * M, MM = M * M, LIST = 256, TPX = QT_R * QT_C;
  __shared__ int3 sl[LIST];
  __shared__ float2 tw[NP];
  __shared__ float2 red[QT_K > 1 ? (QT_K - 1) * 4 * TPX : 1];
  const int tid = threadIdx.x, px = tid % TPX, k = tid / TPX;
  for (int m = tid; m < NP; m += QT_THREADS) tw[m] = g.twn[m];
  const int4 ti = g.qtiles[tile];
  const int R = ti.z + px / QT_C, C = ti.w + px % QT_C;
  float2 acc[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) acc[q] = make_float2(0.f, 0.f);
  for (int b0 = 0; b0 < ti.y; b0 += LIST) {
    const int nb = ti.y - b0 < LIST ? ti.y - b0 : LIST;
    if (b0 > 0) __syncthreads();
    for (int i = tid; i < nb; i += QT_THREADS) {
      const int j = g.qlist[ti.x + b0 + i];
      const int2 pj = g.pos[j];
      sl[i] = make_int3(j, pj.x, pj.y);
    }
    __syncthreads();
#pragma unroll 4
    for (int i = k; i < nb; i += QT_K) {
      const int3 e = sl[i];
      const unsigned rr = (unsigned)(R - e.y), cc = (unsigned)(C - e.z);
      const bool in = rr < (unsigned)M && cc < (unsigned)M;
      // lanes outside the block read its first pixel with zero weights
      const int m1 = in ? (int)rr : 0, m2 = in ? (int)cc : 0;
      const float2* z = g.t + (size_t)e.x * 4 * MM + m1 * M + m2;
      const float2 z00 = z[0], z01 = z[MM], z10 = z[2 * MM], z11 = z[3 * MM];
      const float2* w = g.gw + m1 * NP + m2;
      const float2 zero = make_float2(0.f, 0.f);
      const float2 c0 = in ? w[0] : zero, c1 = in ? w[M] : zero;
      const float2 c2 = in ? w[M * NP] : zero, c3 = in ? w[M * NP + M] : zero;
      const float2 t01 = cmulc(z01, tw[m2]), t10 = cmulc(z10, tw[m1]), t11 = cmulc(z11, tw[m1 + m2]);
      const float2 u0 = cadd(z00, t01), u1 = csub(z00, t01), u2 = cadd(t10, t11), u3 = csub(t10, t11);
      acc[0] = cfma(c0, cadd(u0, u2), acc[0]);
      acc[1] = cfma(c1, cadd(u1, u3), acc[1]);
      acc[2] = cfma(c2, csub(u0, u2), acc[2]);
      acc[3] = cfma(c3, csub(u1, u3), acc[3]);
    }
  }
  if constexpr (QT_K > 1) {
    if (k > 0) {
#pragma unroll
      for (int q = 0; q < 4; ++q) red[((k - 1) * 4 + q) * TPX + px] = acc[q];
    }
    __syncthreads();
    if (k > 0) return;   // no barrier follows
#pragma unroll
    for (int kk = 1; kk < QT_K; ++kk)
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] = cadd(acc[q], red[((kk - 1) * 4 + q) * TPX + px]);
  }
  const size_t npx = (size_t)g.n1 * g.n2;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int Rq = R + M * (q >> 1), Cq = C + M * (q & 1);
    if (Rq < g.n1 && Cq < g.n2) g.part[q * npx + (size_t)Rq * g.n2 + Cq] = cscale(acc[q], 0.25f);
  }
}

template <int M>
__global__ void __launch_bounds__(QT_THREADS) consensus_split(const Recon g, int check_done) {
  if (check_done && *g.done) return;
  consensus_split_body<M>(g, blockIdx.x);
}

// S at one pixel: the partial sums of the quadrants whose base tiles cover
// it, added in the order q = 0..3.
__device__ __forceinline__ float2 split_sum(const Recon& g, int R, int C) {
  const size_t npx = (size_t)g.n1 * g.n2, px = (size_t)R * g.n2 + C;
  const int M = g.np / 2;
  float2 S = make_float2(0.f, 0.f);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int rb = R - M * (q >> 1), cb = C - M * (q & 1);
    if (rb >= 0 && rb < g.qrows && cb >= 0 && cb < g.qcols) S = cadd(S, g.part[q * npx + px]);
  }
  return S;
}

// a9 for the split layout.
__global__ void image_update_split(const Recon g, int check_done) {
  if (check_done && *g.done) return;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n1 * g.n2) return;
  finish_image<kPMACE>(g, i, split_sum(g, i / g.n2, i % g.n2));
}

// After init (mode 0): S of the initial states; after set_state (mode 1):
// also xhat = Lambda^{-1} S (xbar was cleared).
__global__ void image_from_split(const Recon* __restrict__ rec, int mode) {
  const Recon& g = *rec;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n1 * g.n2) return;
  const float2 S = split_sum(g, i / g.n2, i % g.n2);
  g.sold[i] = S;
  if (mode == 1) g.xhat[i] = cscale(S, g.laminv[i]);
}

// The split step of a frame f = d * (patch of img) for block ab at m:
//   W_Np^{a m1 + b m2} sum_q (-1)^{a q1 + b q2} d[m + M q] img[p + m + M q].
// img == nullptr stands for the object 1 + 0i (the default start).
__device__ __forceinline__ float2 split_frame(const Recon& g, int2 pj, int ab, int m1, int m2,
                                              const float2* img) {
  const int M = g.np / 2, a = ab >> 1, b = ab & 1;
  float2 h = make_float2(0.f, 0.f);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int q1 = q >> 1, q2 = q & 1;
    const int r = m1 + M * q1, c = m2 + M * q2;
    const float2 x = img ? img[(size_t)(pj.x + r) * g.n2 + pj.y + c] : make_float2(1.f, 0.f);
    const float2 f = cmul(g.d[r * g.np + c], x);
    h = ((a * q1 + b * q2) & 1) ? csub(h, f) : cadd(h, f);
  }
  return cmul(h, g.twn[a * m1 + b * m2]);
}

// Split-layout states from an object (Alg. 1's initialisation, v_j = P_j x0, stored
// as d v in blocks): element i of block ab of position j.
__global__ void init_split_k(const Recon* __restrict__ rec, const float2* x0) {
  const Recon& g = *rec;
  const int M = g.np / 2, MM = M * M;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)g.J * 4 * MM) return;
  const int j = (int)(i / (4 * MM)), rem = (int)(i - (long long)j * 4 * MM);
  const int ab = rem / MM, m = rem - ab * MM;
  g.t[i] = split_frame(g, g.pos[j], ab, m / M, m % M, x0);
}

// set_state in the split layout: blocks of d v from the given states v.
__global__ void set_state_split_k(const Recon* __restrict__ rec, const float2* __restrict__ v) {
  const Recon& g = *rec;
  const int M = g.np / 2, MM = M * M, np = g.np;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long long)g.J * 4 * MM) return;
  const int j = (int)(i / (4 * MM)), rem = (int)(i - (long long)j * 4 * MM);
  const int ab = rem / MM, m = rem - ab * MM, m1 = m / M, m2 = m % M, a = ab >> 1, b = ab & 1;
  const float2* vj = v + (size_t)j * np * np;
  float2 h = make_float2(0.f, 0.f);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int q1 = q >> 1, q2 = q & 1, k = (m1 + M * q1) * np + m2 + M * q2;
    const float2 f = cmul(g.d[k], vj[k]);
    h = ((a * q1 + b * q2) & 1) ? csub(h, f) : cadd(h, f);
  }
  g.t[i] = cmul(h, g.twn[a * m1 + b * m2]);
}

// get_state in the split layout: v = d^{-1} s + 2 rho P_j xbar with s undone
// from the four blocks.
__global__ void get_state_split_k(const Recon* __restrict__ rec, float2* v) {
  const Recon& g = *rec;
  const int np = g.np, M = np / 2, MM = M * M;
  const long long per = (long long)np * np;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= per * g.J) return;
  const int j = (int)(i / per);
  const int rem = (int)(i - (long long)j * per);
  const int r = rem / np, c = rem - r * np;
  const int m1 = r % M, m2 = c % M, q1 = r / M, q2 = c / M;
  const float2* z = g.t + (size_t)j * 4 * MM + m1 * M + m2;
  float2 s = make_float2(0.f, 0.f);
#pragma unroll
  for (int ab = 0; ab < 4; ++ab) {
    const int a = ab >> 1, b = ab & 1;
    const float2 u = cmulc(z[ab * MM], g.twn[a * m1 + b * m2]);
    s = ((a * q1 + b * q2) & 1) ? csub(s, u) : cadd(s, u);
  }
  const int2 pj = g.pos[j];
  const float2 xb = g.xbar[(size_t)(pj.x + r) * g.n2 + pj.y + c];
  const float2 t = cscale(cmul(g.dinv[rem], cscale(s, 0.25f)), g.np2f);
  v[i] = mann_v(t, xb, g.two_rho);
}

// Data-fit cost of eq. (4) in the split layout: the block ab of F(D P_j xhat)
// per workgroup (frame split as above, M x M forward DFT), against the
// amplitudes of the same coset.
template <int M>
__global__ void __launch_bounds__(M * Geo<M>::A) fit_split(const Recon g, int check_done, int jper) {
  if (check_done && *g.done) return;
  constexpr int A = Geo<M>::A, B = Geo<M>::B, S = M + A, NT = M * A, MB = B / A;
  const int bi = blockIdx.x, slot = bi >> 3;
  const int j = (bi & 7) * jper + (slot >> 2), ab = slot & 3;
  if (j >= g.J) return;
  __shared__ float2 tile[M * S];
  __shared__ float2 tw[M];
  const int tid = threadIdx.x;
  const int2 pj = g.pos[j];
  const int r = tid / A, p = tid % A;
  float2 x[B];
#pragma unroll
  for (int nb = 0; nb < B; ++nb) x[nb] = split_frame(g, pj, ab, r, p + A * nb, g.xhat);
  for (int m = tid; m < M; m += NT) tw[m] = g.twn[2 * m];
  __syncthreads();
  float2* row = tile + r * S;
  row_fwd<M>(x, row, p, tw);
  __syncthreads();
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int ka = 0; ka < A; ++ka) row[p + A * m + B * ka] = x[m * A + ka];
  __syncthreads();
  const int c = tid % M, q = tid / M;
#pragma unroll
  for (int nb = 0; nb < B; ++nb) x[nb] = tile[(q + A * nb) * S + c];
  col_fwd<M>(x, tile, S, c, q, tw);
  const float* yc = g.ys + ((size_t)j * 4 + ab) * M * M + c;
  float acc = 0.f;
#pragma unroll
  for (int m = 0; m < MB; ++m)
#pragma unroll
    for (int ka = 0; ka < A; ++ka)
      acc += fit_term(x[m * A + ka], g.yfac * yc[(size_t)(q + A * m + B * ka) * M]);
  block_sum_to(acc, &g.fit[(size_t)j * 4 + ab], 0.5 / ((double)g.np * g.np));
}

// -------------------------------------------------------------------------
// launchers
// -------------------------------------------------------------------------
static inline unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// Patches per workgroup the whole-patch agent can take for side np: powers
// of two up to 8 within 1024 threads, 1 above Np = 64 (0 for other sides).
int max_ppw(int np) {
  int a = 0;
  switch (np) {
    case 32: a = Geo<32>::A; break;
    case 48: a = Geo<48>::A; break;
    case 64: a = Geo<64>::A; break;
    case 96: case 128: case 160: case 192: case 256: return 1;
    default: return 0;
  }
  int k = 1;
  while (k < 8 && 2 * k * np * a <= 1024) k *= 2;
  return k;
}

int default_ppw(int np) {
  const int k = np == 32 ? PMACE_PPW32 : np == 48 ? PMACE_PPW48 : np == 64 ? PMACE_PPW64 : 1;
  return k <= max_ppw(np) ? k : 1;
}

template <int N, int PPW>
static void small_agent(const Recon& h, hipStream_t st) {
  if constexpr (PPW * N * Geo<N>::A <= 1024) {
    const dim3 grid((h.J + PPW - 1) / PPW), block(PPW * N * Geo<N>::A);
    if (h.method == kSharpPlus)
      hipLaunchKernelGGL((agent_fused<N, kSharpPlus, PPW>), grid, block, 0, st, h);
    else
      hipLaunchKernelGGL((agent_fused<N, kPMACE, PPW>), grid, block, 0, st, h);
  }
}

template <int N>
static hipError_t small_iteration(const Recon& h, int ntiles, hipStream_t st) {
  if constexpr (N <= 64) {
    switch (h.ppw) {
      case 1: small_agent<N, 1>(h, st); break;
      case 2: small_agent<N, 2>(h, st); break;
      case 4: small_agent<N, 4>(h, st); break;
      case 8: small_agent<N, 8>(h, st); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    if (h.ppw != 1) return hipErrorInvalidValue;
    small_agent<N, 1>(h, st);
  }
  if (ntiles > 0) {
    if (h.method == kSharpPlus)
      hipLaunchKernelGGL((consensus_gather<N, true, kSharpPlus>), dim3(ntiles), dim3(GT_THREADS), 0, st, h,
                         0, 0);
    else
      hipLaunchKernelGGL((consensus_gather<N, true, kPMACE>), dim3(ntiles), dim3(GT_THREADS), 0, st, h, 0,
                         0);
  }
  return hipGetLastError();
}

hipError_t launch_small_iteration(int np, const Recon& h, int ntiles, hipStream_t st) {
  switch (np) {
    case 32: return small_iteration<32>(h, ntiles, st);
    case 48: return small_iteration<48>(h, ntiles, st);
    case 64: return small_iteration<64>(h, ntiles, st);
    case 96: return small_iteration<96>(h, ntiles, st);
    case 128: return small_iteration<128>(h, ntiles, st);
    default: return hipErrorInvalidValue;
  }
}

template <int N, int PPW>
static void small_batch_agent(const Recon* recs, const int2* items, int nitems, hipStream_t st) {
  if constexpr (PPW * N * Geo<N>::A <= 1024)
    hipLaunchKernelGGL((agent_fused_batch<N, PPW>), dim3((nitems + PPW - 1) / PPW),
                       dim3(PPW * N * Geo<N>::A), 0, st, recs, items, nitems);
}

template <int N>
static hipError_t small_batch(const Recon* recs, const int2* items, int nitems, const int2* gitems,
                              int ngitems, int ppw, hipStream_t st) {
  if constexpr (N <= 64) {
    switch (ppw) {
      case 1: small_batch_agent<N, 1>(recs, items, nitems, st); break;
      case 2: small_batch_agent<N, 2>(recs, items, nitems, st); break;
      case 4: small_batch_agent<N, 4>(recs, items, nitems, st); break;
      case 8: small_batch_agent<N, 8>(recs, items, nitems, st); break;
      default: return hipErrorInvalidValue;
    }
  } else {
    if (ppw != 1) return hipErrorInvalidValue;
    small_batch_agent<N, 1>(recs, items, nitems, st);
  }
  if (ngitems > 0)
    hipLaunchKernelGGL((consensus_gather_batch<N, true>), dim3(ngitems), dim3(GT_THREADS), 0, st, recs, gitems,
                       0);
  return hipGetLastError();
}

hipError_t launch_small_batch(int np, const Recon* recs, const int2* items, int nitems,
                              const int2* gitems, int ngitems, int ppw, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  if (ppw < 1 || ppw > max_ppw(np)) return hipErrorInvalidValue;
  switch (np) {
    case 32: return small_batch<32>(recs, items, nitems, gitems, ngitems, ppw, st);
    case 48: return small_batch<48>(recs, items, nitems, gitems, ngitems, ppw, st);
    case 64: return small_batch<64>(recs, items, nitems, gitems, ngitems, ppw, st);
    case 96: return small_batch<96>(recs, items, nitems, gitems, ngitems, ppw, st);
    case 128: return small_batch<128>(recs, items, nitems, gitems, ngitems, ppw, st);
    default: return hipErrorInvalidValue;
  }
}

template <int NP>
static void large_iteration(const Recon& h, const Recon* batch_rec, const int2* chunk_tiles,
                            const int2* chunk_rows, hipStream_t st) {
  constexpr int RT = row_threads<NP>(), CT = col_threads<NP>();
  // every position in one chunk: the row consensus finishes a9 itself
  const bool one_chunk = h.chunk >= h.J;
  for (int j0 = 0, g = 0; j0 < h.J; j0 += h.chunk, ++g) {
    const int cnt = (h.J - j0 < h.chunk) ? (h.J - j0) : h.chunk;
    const dim3 rgrid(cnt * (NP / rb_of<NP>())), cgrid(cnt * (NP / CB));
    const int2 ct = chunk_tiles[g];
    if (h.rowspec) {
      // row-spectrum states: rows (window term), columns (new state), then the
      // consensus with the inverse row transforms
      const int2 cr = chunk_rows[g];
      const dim3 crb(cr_threads<NP>()), cg(cr.y);
      if (batch_rec) {
        if (h.nt_stage) {
          hipLaunchKernelGGL((agent_rows_batch<NP, kRowSpec, true>), rgrid, dim3(RT), 0, st, h, j0);
          hipLaunchKernelGGL((agent_cols_batch<NP, kRowSpec, true>), cgrid, dim3(CT), 0, st, h, j0);
        } else {
          hipLaunchKernelGGL((agent_rows_batch<NP, kRowSpec>), rgrid, dim3(RT), 0, st, h, j0);
          hipLaunchKernelGGL((agent_cols_batch<NP, kRowSpec>), cgrid, dim3(CT), 0, st, h, j0);
        }
        if (cr.y > 0 && one_chunk)
          hipLaunchKernelGGL((consensus_rows<NP, true, kRowSpec, true>), cg, crb, 0, st, h, cr.x, j0);
        else if (cr.y > 0)
          hipLaunchKernelGGL((consensus_rows<NP, true, kRowSpec, false>), cg, crb, 0, st, h, cr.x, j0);
      } else if (h.method == kSharpPlus) {
        if (h.nt_stage)
          hipLaunchKernelGGL((agent_rows<NP, kSharpRowSpec, true>), rgrid, dim3(RT), 0, st, h, j0);
        else
          hipLaunchKernelGGL((agent_rows<NP, kSharpRowSpec>), rgrid, dim3(RT), 0, st, h, j0);
        if (h.nt_stage)
          hipLaunchKernelGGL((agent_cols<NP, kSharpRowSpec, true>), cgrid, dim3(CT), 0, st, h, j0);
        else
          hipLaunchKernelGGL((agent_cols<NP, kSharpRowSpec>), cgrid, dim3(CT), 0, st, h, j0);
        if (cr.y > 0 && one_chunk)
          hipLaunchKernelGGL((consensus_rows<NP, false, kSharpRowSpec, true>), cg, crb, 0, st, h, cr.x, j0);
        else if (cr.y > 0)
          hipLaunchKernelGGL((consensus_rows<NP, false, kSharpRowSpec, false>), cg, crb, 0, st, h, cr.x, j0);
      } else {
        if (h.nt_stage) {
          hipLaunchKernelGGL((agent_rows<NP, kRowSpec, true>), rgrid, dim3(RT), 0, st, h, j0);
          hipLaunchKernelGGL((agent_cols<NP, kRowSpec, true>), cgrid, dim3(CT), 0, st, h, j0);
        } else {
          hipLaunchKernelGGL((agent_rows<NP, kRowSpec>), rgrid, dim3(RT), 0, st, h, j0);
          hipLaunchKernelGGL((agent_cols<NP, kRowSpec>), cgrid, dim3(CT), 0, st, h, j0);
        }
        if (cr.y > 0 && one_chunk)
          hipLaunchKernelGGL((consensus_rows<NP, false, kRowSpec, true>), cg, crb, 0, st, h, cr.x, j0);
        else if (cr.y > 0)
          hipLaunchKernelGGL((consensus_rows<NP, false, kRowSpec, false>), cg, crb, 0, st, h, cr.x, j0);
      }
      continue;
    }
    if (batch_rec) {
      hipLaunchKernelGGL((agent_rows_batch<NP, kPMACE>), rgrid, dim3(RT), 0, st, h, j0);
      hipLaunchKernelGGL((agent_cols_batch<NP, kPMACE>), cgrid, dim3(CT), 0, st, h, j0);
      hipLaunchKernelGGL(agent_rowsinv_batch<NP>, rgrid, dim3(RT), 0, st, h, j0);
    } else if (h.method == kSharpPlus) {
      hipLaunchKernelGGL((agent_rows<NP, kSharpPlus>), rgrid, dim3(RT), 0, st, h, j0);
      hipLaunchKernelGGL((agent_cols<NP, kSharpPlus>), cgrid, dim3(CT), 0, st, h, j0);
      hipLaunchKernelGGL((agent_rowsinv<NP, kSharpPlus>), rgrid, dim3(RT), 0, st, h, j0);
    } else {
      hipLaunchKernelGGL((agent_rows<NP, kPMACE>), rgrid, dim3(RT), 0, st, h, j0);
      hipLaunchKernelGGL((agent_cols<NP, kPMACE>), cgrid, dim3(CT), 0, st, h, j0);
      hipLaunchKernelGGL((agent_rowsinv<NP, kPMACE>), rgrid, dim3(RT), 0, st, h, j0);
    }
    if (ct.y > 0) {
      if (batch_rec)
        hipLaunchKernelGGL((consensus_gather_member<NP, false>), dim3(ct.y), dim3(GT_THREADS), 0,
                           st, h, ct.x, j0);
      else if (h.method == kSharpPlus)
        hipLaunchKernelGGL((consensus_gather<NP, false, kSharpPlus>), dim3(ct.y), dim3(GT_THREADS),
                           0, st, h, ct.x, j0);
      else
        hipLaunchKernelGGL((consensus_gather<NP, false, kPMACE>), dim3(ct.y), dim3(GT_THREADS), 0,
                           st, h, ct.x, j0);
    }
  }
  if (h.rowspec && one_chunk) return;
  const unsigned nb = blocks_for((long long)h.n1 * h.n2, 256);
  if (batch_rec)
    hipLaunchKernelGGL(image_update_batch, dim3(nb), dim3(256), 0, st, h);
  else
    hipLaunchKernelGGL(image_update, dim3(nb), dim3(256), 0, st, h);
}

int cr_round(int np) {
  switch (np) {
    case 160: return cr_rows<160>();
    case 192: return cr_rows<192>();
    case 256: return cr_rows<256>();
    default: return 0;
  }
}

hipError_t launch_large_iteration(const Recon& h, const Recon* batch_rec, const int2* chunk_tiles,
                                  const int2* chunk_rows, hipStream_t st) {
  switch (h.np) {
    case 160: large_iteration<160>(h, batch_rec, chunk_tiles, chunk_rows, st); break;
    case 192: large_iteration<192>(h, batch_rec, chunk_tiles, chunk_rows, st); break;
    case 256: large_iteration<256>(h, batch_rec, chunk_tiles, chunk_rows, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// num += the gather of chunk tiles ct (positions from j0 in the stage buffer).
static hipError_t gather_into_num(const Recon& h, int2 ct, int j0, hipStream_t st) {
  if (ct.y <= 0) return hipSuccess;
  switch (h.np) {
#define PMACE_GATHER(N)                                                                           \
  case N:                                                                                         \
    if (h.method == kSharpPlus)                                                                   \
      hipLaunchKernelGGL((consensus_gather<N, false, kSharpPlus>), dim3(ct.y), dim3(GT_THREADS), \
                         0, st, h, ct.x, j0);                                                     \
    else                                                                                          \
      hipLaunchKernelGGL((consensus_gather<N, false, kPMACE>), dim3(ct.y), dim3(GT_THREADS), 0,  \
                         st, h, ct.x, j0);                                                        \
    break;
    PMACE_GATHER(32)
    PMACE_GATHER(48)
    PMACE_GATHER(64)
    PMACE_GATHER(96)
    PMACE_GATHER(128)
    PMACE_GATHER(160)
    PMACE_GATHER(192)
    PMACE_GATHER(256)
#undef PMACE_GATHER
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int M>
static void split_iteration(const Recon& h, int check_done, hipStream_t st) {
  const int jper = (h.J + 7) / 8;
  hipLaunchKernelGGL(agent_split_pair<M>, dim3(8 * jper * 2), dim3(M * Geo<M>::A), 0, st, h, check_done,
                     jper);
  hipLaunchKernelGGL(consensus_split<M>, dim3(h.nqt), dim3(QT_THREADS), 0, st, h, check_done);
  hipLaunchKernelGGL(image_update_split, dim3(blocks_for((long long)h.n1 * h.n2, 256)), dim3(256), 0, st,
                     h, check_done);
}

hipError_t launch_split_iteration(const Recon& h, int check_done, hipStream_t st) {
  switch (h.np) {
    case 128: split_iteration<64>(h, check_done, st); break;
    case 192: split_iteration<96>(h, check_done, st); break;
    case 256: split_iteration<128>(h, check_done, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_split_consensus(const Recon& h, const Recon* rec, int mode, hipStream_t st) {
  switch (h.np) {
    case 128: hipLaunchKernelGGL(consensus_split<64>, dim3(h.nqt), dim3(QT_THREADS), 0, st, h, 0); break;
    case 192: hipLaunchKernelGGL(consensus_split<96>, dim3(h.nqt), dim3(QT_THREADS), 0, st, h, 0); break;
    case 256: hipLaunchKernelGGL(consensus_split<128>, dim3(h.nqt), dim3(QT_THREADS), 0, st, h, 0); break;
    default: return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(image_from_split, dim3(blocks_for((long long)h.n1 * h.n2, 256)), dim3(256), 0, st, rec,
                     mode);
  return hipGetLastError();
}

static hipError_t launch_fit_split(const Recon& h, int check_done, hipStream_t st) {
  const int jper = (h.J + 7) / 8;
  const dim3 grid(8 * jper * 4);
  switch (h.np) {
    case 128: hipLaunchKernelGGL(fit_split<64>, grid, dim3(64 * Geo<64>::A), 0, st, h, check_done, jper); break;
    case 192: hipLaunchKernelGGL(fit_split<96>, grid, dim3(96 * Geo<96>::A), 0, st, h, check_done, jper); break;
    case 256: hipLaunchKernelGGL(fit_split<128>, grid, dim3(128 * Geo<128>::A), 0, st, h, check_done, jper); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Row DFTs of `count` Np x Np patches (in may equal out: each row is read
// whole before it is written): out = scale F_r(in), or scale F_r^*(in).
template <int NP>
static void row_transform(int count, const float2* in, float2* out, bool inverse, float scale,
                          hipStream_t st) {
  const dim3 rgrid(count * (NP / rb_of<NP>()));
  if (inverse)
    hipLaunchKernelGGL((fft_rows<NP, true>), rgrid, dim3(row_threads<NP>()), 0, st, in, out, scale);
  else
    hipLaunchKernelGGL((fft_rows<NP, false>), rgrid, dim3(row_threads<NP>()), 0, st, in, out, scale);
}

static hipError_t launch_row_transform(int np, int count, const float2* in, float2* out, bool inverse,
                                       float scale, hipStream_t st) {
  switch (np) {
    case 160: row_transform<160>(count, in, out, inverse, scale, st); break;
    case 192: row_transform<192>(count, in, out, inverse, scale, st); break;
    case 256: row_transform<256>(count, in, out, inverse, scale, st); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Row-spectrum states from the ones in t (PMACE: probe-weighted): F_r(t)/Np.
static hipError_t states_to_rowspec(const Recon& h, hipStream_t st) {
  return launch_row_transform(h.np, h.J, h.t, h.t, false, 1.f / (float)h.np, st);
}

hipError_t launch_init(const Recon& h, const Recon* rec, const float* z, float scale,
                       int centered, const float2* x0, const int2* chunk_tiles, hipStream_t st) {
  const long long total = (long long)h.J * h.np * h.np;
  const long long npx = (long long)h.n1 * h.n2;
  hipLaunchKernelGGL(init_amplitudes_k, dim3(blocks_for(total, 256)), dim3(256), 0, st, rec, z, scale,
                     centered);
  if (h.split)
    hipLaunchKernelGGL(init_split_k, dim3(blocks_for(total, 256)), dim3(256), 0, st, rec, x0);
  else
    hipLaunchKernelGGL(init_patches_k, dim3(blocks_for(total, 256)), dim3(256), 0, st, rec, x0);
  // Lambda in FP64, accumulated in the (still unused) accumulator image
  double* lam = reinterpret_cast<double*>(h.num);
  hipLaunchKernelGGL(zero_f64_k, dim3(blocks_for(npx, 256)), dim3(256), 0, st, lam, npx);
  for (int j0 = 0, g = 0; j0 < h.J; j0 += h.chunk, ++g)
    if (chunk_tiles[g].y > 0)
      hipLaunchKernelGGL(lambda_gather_k, dim3(chunk_tiles[g].y), dim3(GT_THREADS), 0, st, rec,
                         chunk_tiles[g].x, lam);
  hipLaunchKernelGGL(laminv_k, dim3(blocks_for(npx, 256)), dim3(256), 0, st, rec, lam);
  hipLaunchKernelGGL(init_images_k, dim3(blocks_for(npx, 256)), dim3(256), 0, st, rec, x0);
  if (h.split) return launch_split_consensus(h, rec, 0, st);
  if (h.method == kPMACE) {
    for (int j0 = 0, g = 0; j0 < h.J; j0 += h.chunk, ++g) {
      const hipError_t e = gather_into_num(h, chunk_tiles[g], j0, st);
      if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(sold_from_num, dim3(blocks_for(npx, 256)), dim3(256), 0, st, rec);
  }
  // S above was summed from the stored states themselves
  if (h.rowspec) return states_to_rowspec(h, st);
  return hipGetLastError();
}

hipError_t launch_get_state(const Recon& h, const Recon* rec, float2* v, hipStream_t st) {
  const long long total = (long long)h.J * h.np * h.np;
  if (h.split) {
    hipLaunchKernelGGL(get_state_split_k, dim3(blocks_for(total, 256)), dim3(256), 0, st, rec, v);
  } else if (h.rowspec) {
    // s = F_r^*(H) into v, then v from s in place
    const hipError_t e = launch_row_transform(h.np, h.J, h.t, v, true, 1.f, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(get_state_k, dim3(blocks_for(total, 256)), dim3(256), 0, st, rec,
                       static_cast<const float2*>(v), v);
  } else {
    hipLaunchKernelGGL(get_state_k, dim3(blocks_for(total, 256)), dim3(256), 0, st, rec,
                       static_cast<const float2*>(h.t), v);
  }
  return hipGetLastError();
}

hipError_t launch_set_state(const Recon& h, const Recon* rec, const float2* v,
                            const int2* chunk_tiles, hipStream_t st) {
  const long long npx = (long long)h.n1 * h.n2;
  const long long per = (long long)h.np * h.np;
  hipLaunchKernelGGL(zero_images_k, dim3(blocks_for(npx, 256)), dim3(256), 0, st, rec);
  if (h.split) {
    hipLaunchKernelGGL(set_state_split_k, dim3(blocks_for(per * h.J, 256)), dim3(256), 0, st, rec, v);
    return launch_split_consensus(h, rec, 1, st);
  }
  for (int j0 = 0, g = 0; j0 < h.J; j0 += h.chunk, ++g) {
    const int cnt = (h.J - j0 < h.chunk) ? (h.J - j0) : h.chunk;
    hipLaunchKernelGGL(set_state_k, dim3(blocks_for(cnt * per, 256)), dim3(256), 0, st, rec, v, j0,
                       cnt * per);
    const hipError_t e = gather_into_num(h, chunk_tiles[g], j0, st);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(image_from_num, dim3(blocks_for(npx, 256)), dim3(256), 0, st, rec);
  if (h.method == kSharpPlus) {
    hipLaunchKernelGGL(sharp_image_k, dim3(blocks_for(npx, 256)), dim3(256), 0, st, rec);
    hipLaunchKernelGGL(sharp_state_k, dim3(blocks_for(per * h.J, 256)), dim3(256), 0, st, rec);
  }
  if (h.rowspec) return states_to_rowspec(h, st);
  return hipGetLastError();
}

hipError_t launch_nrmse(const Recon* recs, const int2* ritems, int nritems, const int* fitems, int nf,
                        int update_stop, float tol, int min_iter, hipStream_t st) {
  if (nritems > 0)
    hipLaunchKernelGGL(nrmse_partial, dim3(nritems), dim3(RED_T), 0, st, recs, ritems, update_stop);
  if (nf > 0)
    hipLaunchKernelGGL(nrmse_finish, dim3(nf), dim3(RED_T), 0, st, recs, fitems, update_stop, tol,
                       min_iter);
  return hipGetLastError();
}

template <int NP>
static void fit_large(const Recon& h, const Recon* rec, int check_done, hipStream_t st) {
  for (int j0 = 0; j0 < h.J; j0 += h.chunk) {
    const int cnt = (h.J - j0 < h.chunk) ? (h.J - j0) : h.chunk;
    hipLaunchKernelGGL(fit_rows<NP>, dim3(cnt * (NP / rb_of<NP>())), dim3(row_threads<NP>()), 0, st, rec, j0,
                       check_done);
    hipLaunchKernelGGL(fit_cols<NP>, dim3(cnt * (NP / CB)), dim3(col_threads<NP>()), 0, st, rec, j0,
                       check_done);
  }
}

hipError_t launch_fit_member(const Recon& h, const Recon* rec, int check_done, hipStream_t st) {
  if (h.split) return launch_fit_split(h, check_done, st);
  switch (h.np) {
#define PMACE_FIT(N)                                                                               \
  case N:                                                                                          \
    hipLaunchKernelGGL(fit_small<N>, dim3(h.J), dim3(N * Geo<N>::A), 0, st, rec);                  \
    break;
    PMACE_FIT(32)
    PMACE_FIT(48)
    PMACE_FIT(64)
    PMACE_FIT(96)
    PMACE_FIT(128)
#undef PMACE_FIT
    case 160: fit_large<160>(h, rec, check_done, st); break;
    case 192: fit_large<192>(h, rec, check_done, st); break;
    case 256: fit_large<256>(h, rec, check_done, st); break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fit_batch(int np, const Recon* recs, const int2* items, int nitems, hipStream_t st) {
  if (nitems <= 0) return hipSuccess;
  switch (np) {
#define PMACE_FIT(N)                                                                               \
  case N:                                                                                          \
    hipLaunchKernelGGL(fit_small_batch<N>, dim3(nitems), dim3(N * Geo<N>::A), 0, st, recs, items); \
    break;
    PMACE_FIT(32)
    PMACE_FIT(48)
    PMACE_FIT(64)
    PMACE_FIT(96)
    PMACE_FIT(128)
#undef PMACE_FIT
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_fit_finish(const Recon* recs, const int* fitems, int nf, int update_stop, float tol,
                             int min_iter, hipStream_t st) {
  if (nf > 0)
    hipLaunchKernelGGL(fit_finish, dim3(nf), dim3(RED_T), 0, st, recs, fitems, update_stop, tol,
                       min_iter);
  return hipGetLastError();
}

hipError_t launch_tick(const Recon* recs, const int* fitems, int nf, int max_iter, int cap,
                       hipStream_t st) {
  if (nf > 0)
    hipLaunchKernelGGL(tick_k, dim3(blocks_for(nf, 256)), dim3(256), 0, st, recs, fitems, nf, max_iter,
                       cap);
  return hipGetLastError();
}

template <int NP>
static void fft_large(int count, const float2* in, float2* out, int inverse, hipStream_t st) {
  const float sc = 1.f / sqrtf((float)NP);  // 1/sqrt(NP) per pass
  const dim3 rgrid(count * (NP / rb_of<NP>())), cgrid(count * (NP / CB));
  if (inverse) {
    hipLaunchKernelGGL((fft_cols<NP, true>), cgrid, dim3(col_threads<NP>()), 0, st, in, out, sc);
    hipLaunchKernelGGL((fft_rows<NP, true>), rgrid, dim3(row_threads<NP>()), 0, st, out, out, sc);
  } else {
    hipLaunchKernelGGL((fft_rows<NP, false>), rgrid, dim3(row_threads<NP>()), 0, st, in, out, sc);
    hipLaunchKernelGGL((fft_cols<NP, false>), cgrid, dim3(col_threads<NP>()), 0, st, out, out, sc);
  }
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
    PMACE_FFT_SMALL(48)
    PMACE_FFT_SMALL(64)
    PMACE_FFT_SMALL(96)
    PMACE_FFT_SMALL(128)
#undef PMACE_FFT_SMALL
    case 160: fft_large<160>(count, in, out, inverse, st); break;
    case 192: fft_large<192>(count, in, out, inverse, st); break;
    case 256: fft_large<256>(count, in, out, inverse, st); break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace pmace
