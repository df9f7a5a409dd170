// Register-resident DFT radices and the LDS-exchanged line FFTs used by the
// PMACE kernels (gfx950, wave64).
//
// F in the paper is the 2-D orthonormal DFT (Sec. II).  The kernels compute
// the *unnormalised* transform  X[k] = sum_n x[n] exp(-2 pi i n k / N)  and its
// unnormalised inverse; the 1/Np^2 of a forward+inverse pair is folded into
// the per-pixel probe table, so no pass spends a multiply on scaling.
//
// A line (row or column) of N = A*B points is transformed by A threads with
// one exchange through LDS (Cooley-Tukey, N = A*B):
//   n = n_a + A*n_b,  k = k_b + B*k_a
//   X[k_b + B k_a] = sum_{n_a} W_A^{n_a k_a} W_N^{n_a k_b} sum_{n_b} x[n_a + A n_b] W_B^{n_b k_b}
// Stage 1: thread n_a owns x[n_a + A n_b] (stride A) and does a B-point DFT.
// Twiddle by W_N^{n_a k_b}.  Exchange.  Stage 2: thread p does the A-point
// DFTs for k_b = p, p + A, ... (B/A of them) and ends owning X[k_b + B k_a].
// The inverse runs the same stages backwards, so a forward transform
// followed by a pointwise step and the inverse needs no extra reordering.
#pragma once
#include <hip/hip_runtime.h>

namespace pmace {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// Complex products with their fused multiply-adds written out: the library is
// built with -ffp-contract=off, so every rounding step is the one written
// here, identical in every kernel that inlines it.
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, -(a.y * b.y)), fmaf(a.x, b.y, a.y * b.x));
}
// a * conj(b)
__device__ __forceinline__ float2 cmulc(float2 a, float2 b) {
  return make_float2(fmaf(a.x, b.x, a.y * b.y), fmaf(a.y, b.x, -(a.x * b.y)));
}
// multiply by -i (forward) or +i (inverse)
template <bool INV> __device__ __forceinline__ float2 rotq(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}
// multiply by W_8^1 (forward (1-i)/sqrt2, inverse (1+i)/sqrt2)
template <bool INV> __device__ __forceinline__ float2 w8_1(float2 a) {
  const float s = 0.70710678118654752f;
  return INV ? make_float2((a.x - a.y) * s, (a.x + a.y) * s)
             : make_float2((a.x + a.y) * s, (a.y - a.x) * s);
}
// multiply by W_8^3 (forward (-1-i)/sqrt2, inverse (-1+i)/sqrt2)
template <bool INV> __device__ __forceinline__ float2 w8_3(float2 a) {
  const float s = 0.70710678118654752f;
  return INV ? make_float2((-a.x - a.y) * s, (a.x - a.y) * s)
             : make_float2((a.y - a.x) * s, (-a.x - a.y) * s);
}
// multiply by W_16^k, k compile-time after unrolling
template <bool INV> __device__ __forceinline__ float2 w16(int k, float2 a) {
  const float c1 = 0.92387953251128674f;  // cos(pi/8)
  const float s1 = 0.38268343236508977f;  // sin(pi/8)
  const float sg = INV ? 1.f : -1.f;
  switch (k) {
    case 0: return a;
    case 1: return cmul(a, make_float2(c1, sg * s1));
    case 2: return w8_1<INV>(a);
    case 3: return cmul(a, make_float2(s1, sg * c1));
    case 4: return rotq<INV>(a);
    case 5: return cmul(a, make_float2(-s1, sg * c1));
    case 6: return w8_3<INV>(a);
    default: return cmul(a, make_float2(-c1, sg * s1));
  }
}

// multiply by W_32^k, k compile-time after unrolling (even k: W_16^{k/2})
template <bool INV> __device__ __forceinline__ float2 w32(int k, float2 a) {
  const float c1 = 0.98078528040323044913f;  // cos(pi/16)
  const float s1 = 0.19509032201612826785f;  // sin(pi/16)
  const float c3 = 0.83146961230254523708f;  // cos(3 pi/16)
  const float s3 = 0.55557023301960222474f;  // sin(3 pi/16)
  const float sg = INV ? 1.f : -1.f;
  if (k % 2 == 0) return w16<INV>(k / 2, a);
  switch (k) {
    case 1: return cmul(a, make_float2(c1, sg * s1));
    case 3: return cmul(a, make_float2(c3, sg * s3));
    case 5: return cmul(a, make_float2(s3, sg * c3));
    case 7: return cmul(a, make_float2(s1, sg * c1));
    case 9: return cmul(a, make_float2(-s1, sg * c1));
    case 11: return cmul(a, make_float2(-s3, sg * c3));
    case 13: return cmul(a, make_float2(-c3, sg * s3));
    default: return cmul(a, make_float2(-c1, sg * s1));
  }
}

template <bool INV> __device__ __forceinline__ void dft2(float2* a) {
  float2 t = a[0];
  a[0] = cadd(t, a[1]);
  a[1] = csub(t, a[1]);
}

template <bool INV> __device__ __forceinline__ void dft4r(float2& a0, float2& a1, float2& a2, float2& a3) {
  float2 t0 = cadd(a0, a2), t1 = csub(a0, a2);
  float2 t2 = cadd(a1, a3), t3 = rotq<INV>(csub(a1, a3));
  a0 = cadd(t0, t2);
  a2 = csub(t0, t2);
  a1 = cadd(t1, t3);
  a3 = csub(t1, t3);
}

template <bool INV> __device__ __forceinline__ void dft4(float2* a) { dft4r<INV>(a[0], a[1], a[2], a[3]); }

// 8 points: two 4-point DFTs on even/odd samples, then W_8 butterflies.
template <bool INV> __device__ __forceinline__ void dft8(float2* a) {
  dft4r<INV>(a[0], a[2], a[4], a[6]);
  dft4r<INV>(a[1], a[3], a[5], a[7]);
  float2 o0 = a[1], o1 = w8_1<INV>(a[3]), o2 = rotq<INV>(a[5]), o3 = w8_3<INV>(a[7]);
  float2 e0 = a[0], e1 = a[2], e2 = a[4], e3 = a[6];
  a[0] = cadd(e0, o0); a[4] = csub(e0, o0);
  a[1] = cadd(e1, o1); a[5] = csub(e1, o1);
  a[2] = cadd(e2, o2); a[6] = csub(e2, o2);
  a[3] = cadd(e3, o3); a[7] = csub(e3, o3);
}

// 16 points: two 8-point DFTs on even/odd samples, then W_16 butterflies.
template <bool INV> __device__ __forceinline__ void dft16(float2* a) {
  float2 e[8], o[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) { e[i] = a[2 * i]; o[i] = a[2 * i + 1]; }
  dft8<INV>(e);
  dft8<INV>(o);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    float2 t = w16<INV>(k, o[k]);
    a[k] = cadd(e[k], t);
    a[k + 8] = csub(e[k], t);
  }
}

// 32 points: two 16-point DFTs on even/odd samples, then W_32 butterflies.
template <bool INV> __device__ __forceinline__ void dft32(float2* a) {
  float2 e[16], o[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) { e[i] = a[2 * i]; o[i] = a[2 * i + 1]; }
  dft16<INV>(e);
  dft16<INV>(o);
#pragma unroll
  for (int k = 0; k < 16; ++k) {
    float2 t = w32<INV>(k, o[k]);
    a[k] = cadd(e[k], t);
    a[k + 16] = csub(e[k], t);
  }
}

// 3 points: X1,2 = m -/+ i (sqrt3/2)(a1 - a2) with m = a0 - (a1 + a2)/2
// (signs of i swapped for the inverse).
template <bool INV> __device__ __forceinline__ void dft3r(float2& a0, float2& a1, float2& a2) {
  const float s = 0.86602540378443865f;  // sin(2 pi/3)
  const float2 t = cadd(a1, a2);
  const float2 m = make_float2(fmaf(-0.5f, t.x, a0.x), fmaf(-0.5f, t.y, a0.y));
  const float2 r = rotq<INV>(make_float2(s * (a1.x - a2.x), s * (a1.y - a2.y)));
  a0 = cadd(a0, t);
  a1 = cadd(m, r);
  a2 = csub(m, r);
}

// 5 points, with c_k = cos(2 pi k/5), s_k = sin(2 pi k/5), t1 = a1 + a4,
// t2 = a2 + a3, t3 = a1 - a4, t4 = a2 - a3:
//   X1,4 = (a0 + c1 t1 + c2 t2) -/+ i (s1 t3 + s2 t4)
//   X2,3 = (a0 + c2 t1 + c1 t2) -/+ i (s2 t3 - s1 t4)
template <bool INV> __device__ __forceinline__ void dft5(float2* a) {
  const float c1 = 0.30901699437494742f, c2 = -0.80901699437494742f;
  const float s1 = 0.95105651629515357f, s2 = 0.58778525229247313f;
  const float2 t1 = cadd(a[1], a[4]), t2 = cadd(a[2], a[3]);
  const float2 t3 = csub(a[1], a[4]), t4 = csub(a[2], a[3]);
  const float2 m1 = make_float2(fmaf(c2, t2.x, fmaf(c1, t1.x, a[0].x)), fmaf(c2, t2.y, fmaf(c1, t1.y, a[0].y)));
  const float2 m2 = make_float2(fmaf(c1, t2.x, fmaf(c2, t1.x, a[0].x)), fmaf(c1, t2.y, fmaf(c2, t1.y, a[0].y)));
  const float2 n1 = rotq<INV>(make_float2(fmaf(s1, t3.x, s2 * t4.x), fmaf(s1, t3.y, s2 * t4.y)));
  const float2 n2 = rotq<INV>(make_float2(fmaf(s2, t3.x, -(s1 * t4.x)), fmaf(s2, t3.y, -(s1 * t4.y))));
  a[0] = cadd(a[0], cadd(t1, t2));
  a[1] = cadd(m1, n1);
  a[4] = csub(m1, n1);
  a[2] = cadd(m2, n2);
  a[3] = csub(m2, n2);
}

template <bool INV> __device__ __forceinline__ void dft3(float2* a) { dft3r<INV>(a[0], a[1], a[2]); }

constexpr int inv_mod(int a, int m) {
  for (int x = 1; x < m; ++x)
    if ((a * x) % m == 1) return x;
  return 1;
}

template <int R, bool INV> __device__ __forceinline__ void dft(float2* a);

// N = N1 N2 with gcd(N1, N2) = 1 (Good-Thomas prime-factor map, no
// twiddles): input n = (N2 n1 + N1 n2) mod N, output
// k = (N2 u k1 + N1 v k2) mod N with u = N2^-1 mod N1, v = N1^-1 mod N2, so
// that W_N^{nk} = W_N1^{n1 k1} W_N2^{n2 k2}.
template <int N1, int N2, bool INV> __device__ __forceinline__ void dft_pfa(float2* a) {
  constexpr int N = N1 * N2, U = inv_mod(N2 % N1, N1), V = inv_mod(N1 % N2, N2);
  float2 t[N1][N2];
#pragma unroll
  for (int n1 = 0; n1 < N1; ++n1)
#pragma unroll
    for (int n2 = 0; n2 < N2; ++n2) t[n1][n2] = a[(N2 * n1 + N1 * n2) % N];
#pragma unroll
  for (int n2 = 0; n2 < N2; ++n2) {
    float2 col[N1];
#pragma unroll
    for (int n1 = 0; n1 < N1; ++n1) col[n1] = t[n1][n2];
    dft<N1, INV>(col);
#pragma unroll
    for (int k1 = 0; k1 < N1; ++k1) t[k1][n2] = col[k1];
  }
#pragma unroll
  for (int k1 = 0; k1 < N1; ++k1) dft<N2, INV>(t[k1]);
#pragma unroll
  for (int k1 = 0; k1 < N1; ++k1)
#pragma unroll
    for (int k2 = 0; k2 < N2; ++k2) a[(N2 * U * k1 + N1 * V * k2) % N] = t[k1][k2];
}

template <int R, bool INV> __device__ __forceinline__ void dft(float2* a) {
  if constexpr (R == 2) dft2<INV>(a);
  else if constexpr (R == 3) dft3<INV>(a);
  else if constexpr (R == 4) dft4<INV>(a);
  else if constexpr (R == 5) dft5<INV>(a);
  else if constexpr (R == 8) dft8<INV>(a);
  else if constexpr (R == 12) dft_pfa<3, 4, INV>(a);
  else if constexpr (R == 24) dft_pfa<3, 8, INV>(a);
  else if constexpr (R == 40) dft_pfa<5, 8, INV>(a);
  else if constexpr (R == 32) dft32<INV>(a);
  else { static_assert(R == 16, "radix"); dft16<INV>(a); }
}

// Split N = A*B of a line over A threads with B registers each (B a multiple
// of A).  Powers of two use radix 16/8/4; 48, 96, 192 add a factor 3 and 160
// a factor 5 through the prime-factor DFTs above.
// The splits of 32, 64 and 128 points are build-time choices (tuned):
// 32 = 4x8 or 2x16, 64 = 8x8 or 4x16, 128 = 8x16 or 4x32.
#ifndef PMACE_GEO32_A
#define PMACE_GEO32_A 4
#endif
#ifndef PMACE_GEO64_A
#define PMACE_GEO64_A 8
#endif
#ifndef PMACE_GEO128_A
#define PMACE_GEO128_A 8
#endif
static_assert(PMACE_GEO32_A == 2 || PMACE_GEO32_A == 4, "32-point split");
static_assert(PMACE_GEO64_A == 4 || PMACE_GEO64_A == 8, "64-point split");
static_assert(PMACE_GEO128_A == 4 || PMACE_GEO128_A == 8, "128-point split");
template <int N> struct Geo;
template <> struct Geo<32>  { static constexpr int A = PMACE_GEO32_A, B = 32 / PMACE_GEO32_A; };
template <> struct Geo<48>  { static constexpr int A = 4,  B = 12; };
template <> struct Geo<64>  { static constexpr int A = PMACE_GEO64_A, B = 64 / PMACE_GEO64_A; };
template <> struct Geo<96>  { static constexpr int A = 4,  B = 24; };
template <> struct Geo<128> { static constexpr int A = PMACE_GEO128_A, B = 128 / PMACE_GEO128_A; };
template <> struct Geo<160> { static constexpr int A = 4,  B = 40; };
template <> struct Geo<192> { static constexpr int A = 8,  B = 24; };
template <> struct Geo<256> { static constexpr int A = 16, B = 16; };

// Exchange phases H: the LDS exchange of a line transform moves its B/A
// groups of second-stage inputs in H rounds of B/(H A) groups each, so a
// line needs LDS for N/H points (+ skew) instead of N.  Np = 160 splits only
// as 4 threads x 40 points, and two rounds halve the 320 B of LDS each
// thread would otherwise hold; every other side exchanges in one round.
template <int N> constexpr int exch_phases() { return N == 160 ? 2 : 1; }
// LDS a row-direction line occupies (float2), and the rows a column tile
// needs, with the phases above.
template <int N> constexpr int row_cap() { return N / exch_phases<N>() + Geo<N>::A; }
template <int N> constexpr int col_rows() { return N / exch_phases<N>(); }

// W_N^m = exp(-2 pi i m / N), m = 0..N-1, into LDS from the reconstruction's
// table (computed in FP64 on the host and rounded once).
template <int N> __device__ __forceinline__ void load_twiddles(float2* tw, const float2* twn, int tid,
                                                              int nthreads) {
  for (int m = tid; m < N; m += nthreads) tw[m] = twn[m];
}

// The same table through registers: fetch() issues the loads and store()
// writes them to LDS, so a kernel can issue its own loads in between instead
// of waiting for the table first (the staged passes, whose many workgroups
// each start with that wait).  Every lane loads (an index clamped into the
// table, no branch to wait at); only m < N is written.  The whole-patch
// kernels and the SHARP+ staged passes keep load_twiddles: measured, they
// were slower with it.
template <int N, int NT> struct TwiddleFetch {
  static constexpr int K = (N + NT - 1) / NT;
  float2 v[K];
  __device__ __forceinline__ void fetch(const float2* twn, int tid) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int m = tid + k * NT;
      v[k] = twn[m < N ? m : N - 1];
    }
  }
  __device__ __forceinline__ void store(float2* tw, int tid) const {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const int m = tid + k * NT;
      if (m < N) tw[m] = v[k];
    }
  }
};

// The same values computed in place (FP64 sincospi, rounded once), for the
// standalone transform, which has no workspace.
template <int N> __device__ __forceinline__ void fill_twiddles(float2* tw, int tid, int nthreads) {
  for (int m = tid; m < N; m += nthreads) {
    double s, c;
    sincospi(-2.0 * (double)m / (double)N, &s, &c);
    tw[m] = make_float2((float)c, (float)s);
  }
}

// ---------------------------------------------------------------------------
// Row-direction line FFT.  Thread (r, p), p in [0, A), owns row r of a tile
// whose rows start at row_base (float2 units) with the row exchanged through
// a skewed layout  n_a*(B/H+1) + k_b  (row capacity row_cap<N>() float2),
// one round per exchange phase.
// The A threads of a row are consecutive lanes of one wavefront (A divides
// 64), and only they touch the row's LDS, so the exchange is ordered within
// the wave: a wave's LDS operations execute in order, and wave_sync keeps the
// compiler from moving them across it.  The caller orders any use of the row
// by other waves (the transposes) with workgroup barriers.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// in : x[n_b] = row[p + A n_b]
// out: x[m*A + k_a] = X[(p + A m) + B k_a]
// Round h moves k_b in [h B/H, (h+1) B/H): the groups m in [h M/H, (h+1) M/H)
// read exactly those (k_b = p + A m), and their outputs land in x[m A + k_a],
// the same register range the round has just written out.
template <int N> __device__ __forceinline__ void row_fwd(float2 (&x)[Geo<N>::B], float2* row, int p,
                                                         const float2* tw) {
  constexpr int A = Geo<N>::A, B = Geo<N>::B, M = B / A, H = exch_phases<N>(), BH = B / H, MH = M / H;
  static_assert(64 % A == 0, "a row's threads must share a wavefront");
  static_assert(M % H == 0, "exchange phases must split the groups evenly");
  dft<B, false>(x);
#pragma unroll
  for (int kb = 1; kb < B; ++kb) x[kb] = cmul(x[kb], tw[p * kb]);
#pragma unroll
  for (int h = 0; h < H; ++h) {
    wave_sync();
#pragma unroll
    for (int kb = 0; kb < BH; ++kb) row[p * (BH + 1) + kb] = x[h * BH + kb];
    wave_sync();
#pragma unroll
    for (int m = h * MH; m < (h + 1) * MH; ++m) {
      const int kb = p + A * m - h * BH;
      float2 g[A];
#pragma unroll
      for (int na = 0; na < A; ++na) g[na] = row[na * (BH + 1) + kb];
      dft<A, false>(g);
#pragma unroll
      for (int ka = 0; ka < A; ++ka) x[m * A + ka] = g[ka];
    }
  }
}

// in : x[m*A + k_a] = X[(p + A m) + B k_a]
// out: x[n_b] = unnormalised inverse row[p + A n_b]
template <int N> __device__ __forceinline__ void row_inv(float2 (&x)[Geo<N>::B], float2* row, int p,
                                                         const float2* tw) {
  constexpr int A = Geo<N>::A, B = Geo<N>::B, M = B / A, H = exch_phases<N>(), BH = B / H, MH = M / H;
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int kb = p + A * m;
    dft<A, true>(&x[m * A]);
#pragma unroll
    for (int na = 1; na < A; ++na) x[m * A + na] = cmulc(x[m * A + na], tw[na * kb]);
  }
#pragma unroll
  for (int h = 0; h < H; ++h) {
    wave_sync();
#pragma unroll
    for (int m = h * MH; m < (h + 1) * MH; ++m) {
      const int kb = p + A * m - h * BH;
#pragma unroll
      for (int na = 0; na < A; ++na) row[na * (BH + 1) + kb] = x[m * A + na];
    }
    wave_sync();
#pragma unroll
    for (int kb = 0; kb < BH; ++kb) x[h * BH + kb] = row[p * (BH + 1) + kb];
  }
  dft<B, true>(x);
}

// ---------------------------------------------------------------------------
// Column-direction line FFT.  Thread (c, q), q in [0, A), owns column c of a
// tile with col_rows<N>() rows and row stride S (float2); lanes run along c so
// every LDS access is contiguous across a wave.  The exchange rounds are as
// in the row transforms, ordered by workgroup barriers.
// ---------------------------------------------------------------------------

// in : x[n_b] = col[q + A n_b]
// out: x[m*A + k_a] = X[(q + A m) + B k_a]
template <int N> __device__ __forceinline__ void col_fwd(float2 (&x)[Geo<N>::B], float2* tile, int S,
                                                         int c, int q, const float2* tw) {
  constexpr int A = Geo<N>::A, B = Geo<N>::B, M = B / A, H = exch_phases<N>(), BH = B / H, MH = M / H;
  dft<B, false>(x);
#pragma unroll
  for (int kb = 1; kb < B; ++kb) x[kb] = cmul(x[kb], tw[q * kb]);
#pragma unroll
  for (int h = 0; h < H; ++h) {
    __syncthreads();
#pragma unroll
    for (int kb = 0; kb < BH; ++kb) tile[(kb * A + q) * S + c] = x[h * BH + kb];
    __syncthreads();
#pragma unroll
    for (int m = h * MH; m < (h + 1) * MH; ++m) {
      const int kb = q + A * m - h * BH;
      float2 g[A];
#pragma unroll
      for (int na = 0; na < A; ++na) g[na] = tile[(kb * A + na) * S + c];
      dft<A, false>(g);
#pragma unroll
      for (int ka = 0; ka < A; ++ka) x[m * A + ka] = g[ka];
    }
  }
}

// in : x[m*A + k_a] = X[(q + A m) + B k_a]
// out: x[n_b] = unnormalised inverse col[q + A n_b]
template <int N> __device__ __forceinline__ void col_inv(float2 (&x)[Geo<N>::B], float2* tile, int S,
                                                         int c, int q, const float2* tw) {
  constexpr int A = Geo<N>::A, B = Geo<N>::B, M = B / A, H = exch_phases<N>(), BH = B / H, MH = M / H;
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int kb = q + A * m;
    dft<A, true>(&x[m * A]);
#pragma unroll
    for (int na = 1; na < A; ++na) x[m * A + na] = cmulc(x[m * A + na], tw[na * kb]);
  }
#pragma unroll
  for (int h = 0; h < H; ++h) {
    __syncthreads();
#pragma unroll
    for (int m = h * MH; m < (h + 1) * MH; ++m) {
      const int kb = q + A * m - h * BH;
#pragma unroll
      for (int na = 0; na < A; ++na) tile[(kb * A + na) * S + c] = x[m * A + na];
    }
    __syncthreads();
#pragma unroll
    for (int kb = 0; kb < BH; ++kb) x[h * BH + kb] = tile[(kb * A + q) * S + c];
  }
  dft<B, true>(x);
}

}  // namespace pmace
