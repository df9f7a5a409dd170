// Internal interface between the C ABI (pmace_api.hip) and the kernels
// (pmace_kernels.hip).  Not installed; callers use include/pmace.h.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace pmace {

// Launch-shape parameters.  The defaults are overridden at build time by the
// values the tuner picked (tuned.json beside the package, passed as -D flags).
#ifndef PMACE_GT_K
#define PMACE_GT_K 1      // threads per object pixel in the consensus gather
#endif
#ifndef PMACE_GT_C
#define PMACE_GT_C 64     // consensus gather tile width in object pixels (32 or 64)
#endif
#ifndef PMACE_GATHER_UNROLL
#define PMACE_GATHER_UNROLL 8
#endif
#ifndef PMACE_RB
#define PMACE_RB 16       // Np = 160, 192: patch rows per workgroup in the row passes
#endif
#ifndef PMACE_RB256
#define PMACE_RB256 PMACE_RB  // Np = 256: patch rows per workgroup in the row passes
#endif
#ifndef PMACE_CB
#define PMACE_CB 16       // Np > 128: patch columns per workgroup in the column pass
#endif
#ifndef PMACE_CHUNK256
#define PMACE_CHUNK256 128  // Np > 128: default positions per chunk (at Np = 256)
#endif
#ifndef PMACE_CHUNK256_RS
#define PMACE_CHUNK256_RS 4096  // ... for the row-spectrum agent
#endif
#ifndef PMACE_PPW32
#define PMACE_PPW32 1     // Np = 32: patches per workgroup of the whole-patch agent
#endif
#ifndef PMACE_PPW48
#define PMACE_PPW48 1     // Np = 48
#endif
#ifndef PMACE_PPW64
#define PMACE_PPW64 1     // Np = 64
#endif

// Gather tile of the consensus: GT_R x GT_C object pixels, GT_K threads each
// (GT_R * GT_C * GT_K = 16 GT_C threads per workgroup).  A narrower tile lists
// fewer patches that miss most of its pixels.
constexpr int GT_K = PMACE_GT_K, GT_C = PMACE_GT_C, GT_R = 16 / GT_K;
static_assert(GT_K == 1 || GT_K == 2 || GT_K == 4, "gather split must be 1, 2 or 4");
static_assert(GT_C == 32 || GT_C == 64, "gather tile width must be 32 or 64");
constexpr int GT_THREADS = GT_R * GT_C * GT_K;
static_assert(PMACE_PPW32 >= 1 && PMACE_PPW48 >= 1 && PMACE_PPW64 >= 1, "patches per workgroup");
// Patches per workgroup of the whole-patch agent: the largest the side can
// take (a power of two up to 8 within 1024 threads; 1 for Np = 96, 128; 0 for
// a side without the whole-patch agent), and the build's default (the tuned
// PMACE_PPW<np>, 1 where that exceeds the maximum).  Each patch of a
// workgroup has its own LDS tile and Np * (threads per line) threads.
int max_ppw(int np);
int default_ppw(int np);
// NRMSE reduction: RED_PX object pixels per block of RED_T threads.
constexpr int RED_T = 256, RED_PX = 4096;
// Base tile of the split-layout consensus: QT_R x QT_C pixels, QT_K threads
// each (every QT_K-th entry of the tile's list; partials added in a fixed order).
#ifndef PMACE_QT_K
#define PMACE_QT_K 2
#endif
constexpr int QT_R = 8, QT_C = 32, QT_K = PMACE_QT_K, QT_THREADS = QT_R * QT_C * QT_K;
static_assert(QT_K >= 1 && QT_K <= 4, "split consensus: 1 to 4 threads per pixel");
// Consensus of row-spectrum states: CR_T threads per workgroup, one object
// row segment of CR_W pixels each (CR_W >= 256, so a patch row meets at most
// two segments).
#ifndef PMACE_CR_T
#define PMACE_CR_T 256
#endif
#ifndef PMACE_CR_W
#define PMACE_CR_W 1024
#endif
constexpr int CR_T = PMACE_CR_T, CR_W = PMACE_CR_W;
// Patch rows the row consensus transforms per round for side np (0 if none).
int cr_round(int np);
static_assert(CR_T % 64 == 0 && CR_T <= 1024 && CR_W % CR_T == 0 && CR_W >= 256, "row consensus shape");

// Device-resident description of one reconstruction.  It lives in the
// reconstruction's workspace; batched launches read an array of them.
struct Recon {
  float2* t;            // J*Np*Np   PMACE: d t_j (t_j where d == 0), t_j = v_j - 2 rho w_j,
                        //   v_j = t_j + 2 rho P_j xbar;  SHARP+: t_j (see beta)
  float* ys;            // J*Np*Np   Np*sqrt(z_j)/(1+alpha), DC at [0,0]
  int2* pos;            // J         (row, col) top-left of P_j
  float2* d;            // Np*Np     probe
  float4* pc;           // Np*Np     PMACE: {Re, Im of d^{-1}/Np^2, |d|^kappa, [d == 0]}
  float2* dinv;         // Np*Np     d^{-1}/Np^2, 0 exactly where d == 0 (reading states out)
  float2* gw;           // Np*Np     PMACE consensus weights on the stored states: |d|^kappa / d,
                        //           and |d|^kappa where d == 0 (the state is t there)
  double* omega64;      // Np*Np     the weights in FP64 (SHARP+: |d|^2), for Lambda at init
  float* laminv;        // N1*N2     Lambda^{-1} (0 where Lambda = 0)
  float2* num;          // N1*N2     consensus sum accumulator (Np > 128, set_state)
  float2* sold;         // N1*N2     PMACE: S = sum_j P_j^t |d|^kappa t_j of the current states
  float2* xbar;         // N1*N2     consensus image of the last iteration
  float2* xhat;         // N1*N2     reconstruction (Alg. 1 output, kept by recurrence)
  float2* stage;        // chunk*Np*Np: Np > 128 spectra between passes; SHARP+ (every Np):
                        //   the weighted frames conj(d) P_a s the overlap projection sums
  float2* twn;          // Np       W_Np^m = exp(-2 pi i m/Np), FP64-rounded twiddles
  int4* tiles;          // per gather tile: (list start, count, first row, first col)
  int* tile_list;       // positions overlapping each tile, ascending
  unsigned* status;     // bit0: non-finite consensus image; bit1: bad intensity
  int* done;            // stop flag: nonzero = skip this reconstruction's work
  float2* xref;         // NRMSE reference object, null if none
  unsigned char* mask;  // NRMSE region (nonzero = inside), null = every pixel
  double* red;          // per reduction block: {Re, Im sum conj(xref) xhat, sum |xhat|^2, sum |xref|^2}
  double* track;        // {sum |xref|^2, last nrmse, previous nrmse, iterations counted,
                        //  last data-fit cost, previous data-fit cost}
  double* fit;          // J*fit_bpp per-patch (Np > 128: per column block) data-fit partials
  int n1, n2, np, J;
  float a;              // alpha / (1 + alpha)
  float two_rho;
  float rho;
  int chunk;            // positions per chunk (all J when Np <= 128)
  int n_red;            // NRMSE reduction blocks
  int method;           // 0 PMACE, 1 SHARP+
  float beta;           // SHARP+: beta;  the state is then t with s = t + 2 beta d P_j xbar,
  float ka;             //   two_rho = 2 beta, a = 0, rho = 1, ka = (1 - 2 beta)/Np^2, and
                        //   pc = {conj(d)/Np^2, conj(d)}, laminv = 1/sum P^t |d|^2
  int fit_bpp;          // data-fit partials per patch
  float yfac;           // yfac * ys = Np y_j  (1 + alpha for PMACE, 1 for SHARP+)
  float sb, s2r;        // PMACE: (1 - 2 rho a)/Np^2 and 2 rho/Np^2, the state spectrum
                        //   (X - 2 rho U)/Np^2 = X (sb - s2r ys/|X|)
  float np2f;           // Np^2
  int has_zero;         // the probe has exact zeros (the agent's d == 0 rule applies)
  float cx, co, cn;     // PMACE: xbar' = cx xbar + Lambda^{-1} (co S_old - cn S_new):
                        //   cx = 2 (1 - rho), co = (1 - rho)/rho, cn = 1/rho
  // Split (coset) layout, PMACE with Np = 2M and a probe without zeros: each
  // state is kept as its four blocks Z_ab (a, b in {0, 1}) of the top radix-2
  // step of the transform,
  //   Z_ab[m] = W_Np^{a m1 + b m2} sum_q (-1)^{a q1 + b q2} s[m + M q],  m, q in [0,M)^2 x {0,1}^2,
  // whose M x M DFT is the patch spectrum at the frequencies (2 k1 + a, 2 k2 + b);
  // the amplitudes are stored in the same coset order.
  int split;            // 1: t, ys and the data-fit partials in the split layout
  float2* dr;           // Np^2: 2 rho d (FP64, rounded once), the window weights of the split agent
  float2* part;         // 4 N1 N2: partial consensus sums, one image per quadrant q = 2 q1 + q2
  int4* qtiles;         // per base tile: (list start, count, first row, first col)
  int* qlist;           // positions whose quadrant-0 block meets each base tile, ascending
  int qrows, qcols;     // base tiles cover rows [0, qrows) and columns [0, qcols)
  int nqt;              // number of base tiles
  int ppw;              // Np <= 128: patches per workgroup of the whole-patch agent
  // Row-spectrum states (PMACE, Np > 128, a probe without exact zeros): t holds
  // H_j = F_r(d t_j)/Np, the unnormalised DFT of every row of the probe-weighted
  // state over Np, each row in natural frequency order.  The column pass then
  // writes the new state directly, and the consensus inverts the rows.
  int rowspec;
  // Row-spectrum agent: when a chunk's stage is over twice the 256 MB
  // Infinity Cache, the row pass writes it, and the column pass the new
  // states (PMACE and SHARP+), with non-temporal stores (smaller stages gain
  // from the cache on their way to the column pass)
  int nt_stage;
  int4* citems;         // per (chunk, object row, segment): (list start, count, row, first column)
  int4* clist;          // per entry: (j, row of P_j on that object row, patch column, 0), ascending j
};

// Kernel launchers (stream-ordered; return the hipError_t of the launches).
// `rec` / `recs` are device addresses of Recon descriptors, `h` a host copy.
// PMACE also forms S of the initial states (per chunk, chunk_tiles as below).
hipError_t launch_init(const Recon& h, const Recon* rec, const float* z, float scale, int centered,
                       const float2* x0, const int2* chunk_tiles, hipStream_t st);
// Np <= 128, one reconstruction: fused agent over its J positions, then the
// fused gather + image update over its ntiles tiles.
hipError_t launch_small_iteration(int np, const Recon& h, int ntiles, hipStream_t st);
// Np <= 128, batched: agent over `items` (recon index, position), ppw of them
// per workgroup, and the fused gather + image update over `gitems` (recon
// index, tile).
hipError_t launch_small_batch(int np, const Recon* recs, const int2* items, int nitems,
                              const int2* gitems, int ngitems, int ppw, hipStream_t st);
// Np > 128, one reconstruction, chunk by chunk; chunk_tiles[g] = (first tile,
// tile count) of chunk g (host array); the descriptor h passed by value.
// batch_rec non-null: run as a batch member (its kernels honour the stop
// flag).
// h.rowspec: chunk_rows[g] = (first row item, count) of chunk g (host array).
hipError_t launch_large_iteration(const Recon& h, const Recon* batch_rec, const int2* chunk_tiles,
                                  const int2* chunk_rows, hipStream_t st);
hipError_t launch_get_state(const Recon& h, const Recon* rec, float2* v, hipStream_t st);
hipError_t launch_set_state(const Recon& h, const Recon* rec, const float2* v,
                            const int2* chunk_tiles, hipStream_t st);
// a10: NRMSE of xhat against xref for the reconstructions in `ritems`
// (recon index, reduction block); `fitems` lists the recon indices to finish.
// With update_stop, a member whose NRMSE changed by less than tol once
// min_iter iterations have been counted is stopped.
hipError_t launch_nrmse(const Recon* recs, const int2* ritems, int nritems, const int* fitems,
                        int nf, int update_stop, float tol, int min_iter, hipStream_t st);
// Data-fit cost of eq. (4) at xhat: partials of one reconstruction (all Np;
// rec = its device descriptor, check_done: skip if stopped), or of the
// batched Np <= 128 positions `items` (recon index, position).
hipError_t launch_fit_member(const Recon& h, const Recon* rec, int check_done, hipStream_t st);
hipError_t launch_fit_batch(int np, const Recon* recs, const int2* items, int nitems, hipStream_t st);
// Sum the partials: with update_stop into track[4] (previous value to
// track[5]), stopping members whose cost changed by at most tol (relative);
// without, into track[6] only.
hipError_t launch_fit_finish(const Recon* recs, const int* fitems, int nf, int update_stop, float tol,
                             int min_iter, hipStream_t st);
// cap = 0: count one iteration for each running member (before the stop
// rule is evaluated); cap = 1: stop running members that reached max_iter.
hipError_t launch_tick(const Recon* recs, const int* fitems, int nf, int max_iter, int cap,
                       hipStream_t st);
hipError_t launch_fft2(int np, int count, const float2* in, float2* out, int inverse, hipStream_t st);
// Split layout (h.split): one iteration (agent on every (position, coset),
// consensus over the base tiles, image update), the descriptor h passed by
// value; check_done: skip if the stop flag is set (batch members).
hipError_t launch_split_iteration(const Recon& h, int check_done, hipStream_t st);
// Split layout: the consensus sum of the current states into part, then
// mode 0: sold = S (after init), mode 1: xhat = Lambda^{-1} S and sold = S
// (after set_state).
hipError_t launch_split_consensus(const Recon& h, const Recon* rec, int mode, hipStream_t st);

}  // namespace pmace
