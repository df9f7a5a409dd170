// C ABI of libpmace.so (declared in include/pmace.h).
//
// Host responsibilities: argument validation, the workspace layout, the FP64
// tables computed once per reconstruction (|d|^kappa, d^{-1}, Lambda^{-1} of
// eq. (11)), the consensus tile tables, and replaying iterations as HIP
// graphs (one per reconstruction, one per batch).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <cstring>
#include <new>
#include <utility>
#include <vector>

#include "pmace.h"
#include "pmace_internal.hpp"

using pmace::Recon;

namespace {

constexpr size_t kAlign = 256;
// Patch sides run by the fused one-workgroup agent; larger ones (160, 192,
// 256) by the three-pass agent.
constexpr int kSmallNp[] = {32, 48, 64, 96, 128};
constexpr int kClasses = 5;
inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

bool graphs_enabled() {
  const char* e = std::getenv("PMACE_NO_GRAPH");
  return !(e && e[0] == '1');
}

// A stream-ordered iteration captured once and replayed.
struct Graph {
  hipGraph_t g = nullptr;
  hipGraphExec_t x = nullptr;
  void release() {
    if (x) (void)hipGraphExecDestroy(x);
    if (g) (void)hipGraphDestroy(g);
    x = nullptr;
    g = nullptr;
  }
};

}  // namespace

struct pmace_ctx {
  pmace_params prm;
  hipStream_t stream;
  int device;
  Recon h;                        // host copy of the device descriptor
  Recon* dev;                     // device descriptor (in the workspace)
  int2* items;                    // device: (0, j) agent work items
  int2* gitems;                   // device: (0, tile) gather work items
  int2* ritems;                   // device: (0, b) NRMSE reduction items
  int* fitem;                     // device: {0}
  int ngitems;
  std::vector<int2> chunk_tiles;  // host: per chunk (first gather item, count)
  std::vector<int2> chunk_rows;   // host, row-spectrum states: per chunk (first row item, count)
  Graph graph;                    // one iteration
  Graph graph_k;                  // kGraphIters iterations back to back
  bool graph_tried;
  pmace_status sticky;            // first asynchronous failure seen
  unsigned long long resets;      // times the host cleared the stop flag
  // batches holding a copy of this context's descriptor (and its index there):
  // pmace_set_reference updates those copies too
  std::vector<std::pair<pmace_batch*, int>> holders;
};

struct pmace_batch {
  int n;
  hipStream_t stream;
  std::vector<pmace_ctx*> ctxs;
  Recon* recs;                 // device: member descriptors
  int2* items[kClasses];       // device: agent items per fused patch size (kSmallNp)
  int nitems[kClasses];
  int ppw[kClasses];           // patches per workgroup of each class's merged agent launch
  int2* gitems[kClasses];      // device: gather items per class
  int ngitems[kClasses];
  int2* ritems;                // device: (member, block) NRMSE items
  int nritems;
  int* fitems;                 // device: member indices
  pmace_stop_rule rule;
  hipStream_t lanes[4];
  hipEvent_t fork, join[4];
  Graph graph;                 // one iteration
  Graph graph_check;           // one iteration + stop-rule evaluation
  bool graph_tried;
  long long iters;             // iterations launched by this batch
  int step_calls;              // pmace_batch_step calls so far
  // Np > 128 members a poll found stopped: their kernel chains are left out
  // of the launches (they would only read the flag and exit), until the host
  // clears the member's flag (pmace_iterate, pmace_set_reference), seen as a
  // change of its reset count from the one recorded here.
  std::vector<char> pruned;
  std::vector<unsigned long long> pruned_at;
};

namespace {

bool np_supported(int np) {
  for (int s : kSmallNp)
    if (np == s) return true;
  return np == 160 || np == 192 || np == 256;
}
bool np_large(int np) { return np > 128; }

bool rowspec_allowed(const pmace_params& p);

// Positions per chunk: Np <= 128 runs all positions in one fused launch;
// Np > 128 stages chunk*Np^2 spectra between its passes.
int chunk_of(const pmace_params& p) {
  int c = p.num_pos;
  // default: the tuned bound for 256-point patches (one for the three-pass
  // agent, one for the row-spectrum agent), scaled so that every patch side
  // stages about the same bytes per chunk
  if (np_large(p.np)) {
    const long long c256 = rowspec_allowed(p) ? PMACE_CHUNK256_RS : PMACE_CHUNK256;
    c = p.chunk > 0 ? p.chunk : (int)(c256 * 256 * 256 / ((long long)p.np * p.np));
  }
  if (c > p.num_pos) c = p.num_pos;
  // the same number of chunks, evened out (no small last chunk)
  const int n = (p.num_pos + c - 1) / c;
  return (p.num_pos + n - 1) / n;
}
int num_chunks(const pmace_params& p) {
  const int c = chunk_of(p);
  return (p.num_pos + c - 1) / c;
}
// Upper bounds of the gather tables (depend on sizes only, not on positions).
size_t max_tiles(const pmace_params& p) {
  return (size_t)num_chunks(p) * ((p.n1 + pmace::GT_R - 1) / pmace::GT_R) *
         ((p.n2 + pmace::GT_C - 1) / pmace::GT_C);
}
size_t max_list(const pmace_params& p) {
  return (size_t)p.num_pos * ((p.np - 1) / pmace::GT_R + 2) * ((p.np - 1) / pmace::GT_C + 2);
}
int num_red(const pmace_params& p) {
  return (int)(((size_t)p.n1 * p.n2 + pmace::RED_PX - 1) / pmace::RED_PX);
}

pmace_status check_params(const pmace_params* p) {
  if (!p) return PMACE_EINVAL;
  if (p->np < 1 || p->num_pos < 1 || p->n1 < p->np || p->n2 < p->np) return PMACE_EINVAL;
  if (!(std::isfinite(p->alpha) && p->alpha >= 0.f)) return PMACE_EINVAL;
  if (!(std::isfinite(p->kappa) && p->kappa >= 0.f)) return PMACE_EINVAL;
  if (!(std::isfinite(p->rho) && p->rho > 0.f && p->rho < 1.f)) return PMACE_EINVAL;
  constexpr uint32_t kAgents = PMACE_STAGED_AGENT | PMACE_SPLIT_AGENT | PMACE_ROWSPEC_AGENT;
  if (p->flags & ~(PMACE_CENTERED_DC | kAgents)) return PMACE_EINVAL;
  const uint32_t ag = p->flags & kAgents;
  if (ag & (ag - 1)) return PMACE_EINVAL;  // at most one agent asked for
  if (p->chunk < 0) return PMACE_EINVAL;
  if (p->method != PMACE_METHOD_PMACE && p->method != PMACE_METHOD_SHARP_PLUS) return PMACE_EINVAL;
  if (p->method == PMACE_METHOD_SHARP_PLUS && !(std::isfinite(p->beta) && p->beta >= 0.f && p->beta <= 1.f))
    return PMACE_EINVAL;
  if ((long long)p->n1 * p->n2 > (1LL << 30)) return PMACE_EINVAL;
  if (!np_supported(p->np)) return PMACE_EUNSUPPORTED;
  if (p->ppw < 0 || (p->ppw > 0 && ((p->ppw & (p->ppw - 1)) != 0 || p->ppw > pmace::max_ppw(p->np))))
    return PMACE_EINVAL;
  return PMACE_OK;
}

// Section offsets inside the workspace (relative to the aligned base).
struct Layout {
  size_t t, ys, pos, d, pc, dinv, gw, omega64, laminv, num, sold, xbar, xhat, stage, tiles, list, status, desc,
      items, gitems, ritems, red, tw, fit, dr, qtiles, qlist, citems, clist, total;
};

// Patch sides whose default agent is the split (coset-block) one: a build
// choice measured by the tuner (bit 0: Np = 128, bit 1: 192, bit 2: 256).
#ifndef PMACE_SPLIT_SIDES
#define PMACE_SPLIT_SIDES 2
#endif
bool split_default(int np) {
  const int bit = np == 128 ? 1 : np == 192 ? 2 : np == 256 ? 4 : 0;
  return (PMACE_SPLIT_SIDES & bit) != 0;
}
// The split agent may run: PMACE with Np in {128, 192, 256} when asked for,
// or by default where the build chose it, unless the other agent is asked
// for.  Whether it does also needs a probe without exact zeros (known at init).
bool split_allowed(const pmace_params& p) {
  if (p.method != PMACE_METHOD_PMACE) return false;
  if (p.np != 128 && p.np != 192 && p.np != 256) return false;
  if (p.flags & PMACE_SPLIT_AGENT) return true;
  if (p.flags & (PMACE_STAGED_AGENT | PMACE_ROWSPEC_AGENT)) return false;
  return split_default(p.np);
}
// Patch sides whose default agent keeps row-spectrum states (bit 0: Np = 160,
// bit 1: 192, bit 2: 256), where the split agent is not the default: a build
// choice measured by the tuner.
#ifndef PMACE_ROWSPEC_SIDES
#define PMACE_ROWSPEC_SIDES 0
#endif
bool rowspec_default(int np) {
  const int bit = np == 160 ? 1 : np == 192 ? 2 : np == 256 ? 4 : 0;
  return (PMACE_ROWSPEC_SIDES & bit) != 0;
}
// SHARP+ on the row-spectrum agent by default where PMACE is (1), or only
// when asked for (0): a build choice measured by the tuner.
#ifndef PMACE_ROWSPEC_SHARP
#define PMACE_ROWSPEC_SHARP 0
#endif
// The row-spectrum agent may run: Np > 128 when asked for, or by default
// where the build chose it and no other agent is asked for or chosen.  PMACE
// also needs a probe without exact zeros (known at init; its d = 0 rule acts
// per pixel); SHARP+ has no such rule.
bool rowspec_allowed(const pmace_params& p) {
  if (!np_large(p.np)) return false;
  if (p.flags & PMACE_ROWSPEC_AGENT) return true;
  if (p.flags & (PMACE_STAGED_AGENT | PMACE_SPLIT_AGENT)) return false;
  if (p.method == PMACE_METHOD_SHARP_PLUS && !PMACE_ROWSPEC_SHARP) return false;
  return !split_allowed(p) && rowspec_default(p.np);
}
// Bounds of its consensus tables (sizes only): every (chunk, object row,
// segment) item, and an entry per patch row and segment it meets (at most two,
// as a segment is at least 256 wide).
int cr_segments(const pmace_params& p) { return (p.n2 + pmace::CR_W - 1) / pmace::CR_W; }
size_t cr_items(const pmace_params& p) { return (size_t)num_chunks(p) * p.n1 * cr_segments(p); }
size_t cr_list(const pmace_params& p) { return (size_t)p.num_pos * p.np * std::min(2, cr_segments(p)); }
// Base tiles of the split consensus: rows [0, qrows), columns [0, qcols), the
// quadrant-0 blocks of all positions lie in [0, n1 - M) x [0, n2 - M).
int split_rows(const pmace_params& p) {
  const int M = p.np / 2;
  return (p.n1 - M + pmace::QT_R - 1) / pmace::QT_R * pmace::QT_R;
}
int split_cols(const pmace_params& p) {
  const int M = p.np / 2;
  return (p.n2 - M + pmace::QT_C - 1) / pmace::QT_C * pmace::QT_C;
}
size_t split_tiles(const pmace_params& p) {
  return (size_t)(split_rows(p) / pmace::QT_R) * (split_cols(p) / pmace::QT_C);
}
size_t split_list(const pmace_params& p) {
  const int M = p.np / 2;
  return (size_t)p.num_pos * ((M - 1) / pmace::QT_R + 2) * ((M - 1) / pmace::QT_C + 2);
}

// Stage buffer: Np > 128 keeps a chunk's spectra between its passes; SHARP+
// keeps its overlap numerators there; PMACE with Np <= 128 needs none.
size_t stage_patches(const pmace_params& p) {
  if (np_large(p.np)) return (size_t)chunk_of(p);
  return p.method == PMACE_METHOD_SHARP_PLUS ? (size_t)chunk_of(p) : 0;
}

// Data-fit partial sums per patch: one, or one per column block for Np > 128.
int fit_bpp(const pmace_params& p) { return np_large(p.np) ? p.np / PMACE_CB : 1; }

// Launch order of one row of tiles t[first, end), left to right. The
// dispatcher sends workgroup b to XCD b mod 8, and each XCD has its own L2.
// Side-by-side tiles read the same state lines at their common edge, so slot
// b gets tile (b mod 8) * q + b / 8 of the row (q = n / 8; the last n mod 8
// stay in place): each XCD runs q side-by-side tiles of every row, and the
// second read of an edge line hits its L2. Only which workgroup sums which
// pixel changes; every pixel's sum is the same.
void xcd_runs(std::vector<int4>& t, size_t first, size_t end) {
  const size_t q = (end - first) / 8;
  if (q == 0) return;
  const std::vector<int4> row(t.begin() + first, t.begin() + first + 8 * q);
  for (size_t b = 0; b < 8 * q; ++b) t[first + b] = row[(b % 8) * q + b / 8];
}

Layout layout_of(const pmace_params& p) {
  Layout L;
  const size_t P = (size_t)p.num_pos * p.np * p.np;
  const size_t npx = (size_t)p.n1 * p.n2;
  const size_t np2 = (size_t)p.np * p.np;
  size_t o = 0;
  L.t = o;       o = align_up(o + P * 8);
  L.ys = o;      o = align_up(o + P * 4);
  L.pos = o;     o = align_up(o + (size_t)p.num_pos * 8);
  L.d = o;       o = align_up(o + np2 * 8);
  L.pc = o;      o = align_up(o + np2 * 16);
  L.dinv = o;    o = align_up(o + np2 * 8);
  L.gw = o;      o = align_up(o + np2 * 8);
  L.omega64 = o; o = align_up(o + np2 * 8);
  L.laminv = o;  o = align_up(o + npx * 4);
  L.num = o;     o = align_up(o + npx * 8);
  L.sold = o;    o = align_up(o + npx * 8);
  L.xbar = o;    o = align_up(o + npx * 8);
  L.xhat = o;    o = align_up(o + npx * 8);
  // the staged spectra and the split layout's partial sums never coexist
  const bool sp = split_allowed(p);
  L.stage = o;   o = align_up(o + std::max(stage_patches(p) * np2 * 8, sp ? 4 * npx * 8 : (size_t)0));
  L.tiles = o;   o = align_up(o + max_tiles(p) * 16);
  L.list = o;    o = align_up(o + max_list(p) * 4);
  L.status = o;  o = align_up(o + 128);  // status word, stop flag, finish item, track[8] at +32
  L.desc = o;    o = align_up(o + sizeof(Recon));
  L.items = o;   o = align_up(o + (size_t)p.num_pos * 8);
  L.gitems = o;  o = align_up(o + max_tiles(p) * 8);
  L.ritems = o;  o = align_up(o + (size_t)num_red(p) * 8);
  L.red = o;     o = align_up(o + (size_t)num_red(p) * 32);
  L.tw = o;      o = align_up(o + 256 * 8);
  L.fit = o;     o = align_up(o + (size_t)p.num_pos * std::max(fit_bpp(p), sp ? 4 : 0) * 8);
  L.dr = o;      o = align_up(o + (sp ? np2 * 8 : 0));
  L.qtiles = o;  o = align_up(o + (sp ? split_tiles(p) * 16 : 0));
  L.qlist = o;   o = align_up(o + (sp ? split_list(p) * 4 : 0));
  const bool rs = rowspec_allowed(p);
  L.citems = o;  o = align_up(o + (rs ? cr_items(p) * 16 : 0));
  L.clist = o;   o = align_up(o + (rs ? cr_list(p) * 16 : 0));
  L.total = o;
  return L;
}

#define PM_HIP(call)                            \
  do {                                          \
    hipError_t e_ = (call);                     \
    if (e_ != hipSuccess) return PMACE_EDEVICE; \
  } while (0)

pmace_status record(pmace_ctx* c, pmace_status s) {
  if (s != PMACE_OK && c->sticky == PMACE_OK) c->sticky = s;
  return s;
}

// A member that runs as its own chain of kernels (three-pass or split agent).
bool own_chain(const pmace_ctx* c) { return np_large(c->prm.np) || c->h.split; }

pmace_status enqueue_iteration(pmace_ctx* c, hipStream_t st) {
  if (c->h.split)
    PM_HIP(pmace::launch_split_iteration(c->h, 0, st));
  else if (np_large(c->prm.np))
    PM_HIP(pmace::launch_large_iteration(c->h, nullptr, c->chunk_tiles.data(), c->chunk_rows.data(), st));
  else
    PM_HIP(pmace::launch_small_iteration(c->prm.np, c->h, c->ngitems, st));
  return PMACE_OK;
}

// Capture `body(stream)` into g (on a private capture stream; the graph is
// then launched on the caller's stream).
template <class F>
pmace_status capture(Graph& g, F body) {
  hipStream_t cs = nullptr;
  PM_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  pmace_status s = PMACE_OK;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    s = PMACE_EDEVICE;
  } else {
    s = body(cs);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &graph);
    if (s == PMACE_OK && (e != hipSuccess || !graph)) s = PMACE_EDEVICE;
    if (s == PMACE_OK && hipGraphInstantiate(&g.x, graph, nullptr, nullptr, 0) != hipSuccess)
      s = PMACE_EDEVICE;
    g.g = graph;
    if (s != PMACE_OK) g.release();
  }
  (void)hipStreamDestroy(cs);
  return s;
}

// Reset the stop flag and the NRMSE history of a reconstruction.
__global__ void reset_tracking_k(int* done, double* track) {
  *done = 0;
  track[0] = 0.0;
  track[1] = __builtin_inf();
  track[2] = __builtin_inf();
  track[3] = 0.0;
  track[4] = __builtin_inf();
  track[5] = __builtin_inf();
  track[6] = __builtin_inf();
}

// Copy a member's host descriptor into a batch's descriptor array.
hipError_t batch_recs_update(pmace_batch* b, int i, const Recon& h, hipStream_t st);
// Drop a destroyed member's entry from a batch (the batch can then only be destroyed).
void batch_forget(pmace_batch* b, int i);

}  // namespace

extern "C" {

const char* pmace_status_str(pmace_status s) {
  switch (s) {
    case PMACE_OK: return "ok";
    case PMACE_EINVAL: return "invalid argument";
    case PMACE_EUNSUPPORTED: return "unsupported configuration";
    case PMACE_ENOMEM: return "workspace too small";
    case PMACE_EDEVICE: return "HIP device error";
    case PMACE_ESTATE: return "invalid context state";
    case PMACE_EDIVERGED: return "consensus image not finite";
  }
  return "unknown status";
}

size_t pmace_footprint(const pmace_params* p) {
  if (check_params(p) != PMACE_OK) return 0;
  return layout_of(*p).total + kAlign;  // slack to align an arbitrary base
}

pmace_status pmace_init(const pmace_params* params, const void* probe_d, const int32_t* pos_d,
                        const float* intensity_d, const void* x0_d, void* workspace_d,
                        size_t ws_bytes, void* hip_stream, pmace_ctx** out) {
  if (!out) return PMACE_EINVAL;
  *out = nullptr;
  pmace_status ps = check_params(params);
  if (ps != PMACE_OK) return ps;
  if (!probe_d || !pos_d || !intensity_d || !workspace_d) return PMACE_EINVAL;
  const pmace_params p = *params;
  if (ws_bytes < pmace_footprint(&p)) return PMACE_ENOMEM;
  hipStream_t st = reinterpret_cast<hipStream_t>(hip_stream);

  const int np = p.np, J = p.num_pos, n1 = p.n1, n2 = p.n2;
  const size_t np2 = (size_t)np * np, npx = (size_t)n1 * n2;

  // Small inputs come to the host for validation and the FP64 tables.
  std::vector<std::complex<float>> probe(np2);
  std::vector<int32_t> pos(2 * (size_t)J);
  PM_HIP(hipMemcpyAsync(probe.data(), probe_d, np2 * 8, hipMemcpyDeviceToHost, st));
  PM_HIP(hipMemcpyAsync(pos.data(), pos_d, (size_t)J * 8, hipMemcpyDeviceToHost, st));
  PM_HIP(hipStreamSynchronize(st));
  for (int j = 0; j < J; ++j) {
    const int r = pos[2 * j], c = pos[2 * j + 1];
    if (r < 0 || c < 0 || r > n1 - np || c > n2 - np) return PMACE_EINVAL;
  }
  for (auto& v : probe)
    if (!std::isfinite(v.real()) || !std::isfinite(v.imag())) return PMACE_EINVAL;

  // |d|^kappa, d^{-1} (scaled by 1/Np^2: the unnormalised forward+inverse
  // DFT pair), the d == 0 mask, and Lambda^{-1} (0 where Lambda = 0).
  // SHARP+ (eq. (15)): weights conj(d) over the normaliser sum_k P_k^t |d|^2.
  const bool sharp = p.method == PMACE_METHOD_SHARP_PLUS;
  std::vector<float> pc(4 * np2), gw(2 * np2, 0.f), dinv(2 * np2, 0.f);
  bool has_zero = false;
  std::vector<double> omega(np2);
  const double inv_np2 = 1.0 / ((double)np * np);
  for (size_t i = 0; i < np2; ++i) {
    const std::complex<double> dd(probe[i].real(), probe[i].imag());
    const double mag = std::abs(dd);
    if (sharp) {
      omega[i] = mag * mag;
      pc[4 * i + 0] = (float)(dd.real() * inv_np2);
      pc[4 * i + 1] = (float)(-dd.imag() * inv_np2);
      pc[4 * i + 2] = (float)dd.real();
      pc[4 * i + 3] = (float)(-dd.imag());
      continue;
    }
    omega[i] = std::pow(mag, (double)p.kappa);
    std::complex<double> di(0.0, 0.0);
    if (mag != 0.0) {
      di = inv_np2 / dd;
      const std::complex<double> w = omega[i] / dd;  // weights on the stored d t
      gw[2 * i + 0] = (float)w.real();
      gw[2 * i + 1] = (float)w.imag();
    } else {
      has_zero = true;   // the stored state is t itself there: weight |d|^kappa (1 if kappa = 0)
      gw[2 * i + 0] = (float)omega[i];
    }
    pc[4 * i + 0] = (float)di.real();
    pc[4 * i + 1] = (float)di.imag();
    dinv[2 * i + 0] = pc[4 * i + 0];
    dinv[2 * i + 1] = pc[4 * i + 1];
    // d != 0 must not round to the d == 0 marker: keep the smallest subnormal
    if (mag != 0.0 && dinv[2 * i] == 0.f && dinv[2 * i + 1] == 0.f) dinv[2 * i] = 1e-45f;
    pc[4 * i + 2] = (float)omega[i];
    pc[4 * i + 3] = mag == 0.0 ? 1.f : 0.f;
  }
  // Lambda = sum_j P_j^t omega and its inverse are formed on the device from
  // the FP64 weights and the consensus tile lists (see launch_init).

  // Split layout: the window weights 2 rho d (FP64, rounded once) and the
  // base tiles of its consensus.
  const bool split = split_allowed(p) && !has_zero;
  const int M = np / 2;
  std::vector<float> dr;
  std::vector<int4> qtiles;
  std::vector<int> qlist;
  if (split) {
    dr.assign(2 * np2, 0.f);
    for (size_t i = 0; i < np2; ++i) {
      dr[2 * i] = (float)(2.0 * (double)p.rho * (double)probe[i].real());
      dr[2 * i + 1] = (float)(2.0 * (double)p.rho * (double)probe[i].imag());
    }
    const int qr = split_rows(p) / pmace::QT_R, qc = split_cols(p) / pmace::QT_C;
    std::vector<std::vector<int>> per_tile((size_t)qr * qc);
    for (int j = 0; j < J; ++j) {
      const int r = pos[2 * j], cc = pos[2 * j + 1];
      for (int tr = r / pmace::QT_R; tr <= (r + M - 1) / pmace::QT_R && tr < qr; ++tr)
        for (int tc = cc / pmace::QT_C; tc <= (cc + M - 1) / pmace::QT_C && tc < qc; ++tc)
          per_tile[(size_t)tr * qc + tc].push_back(j);
    }
    for (int tr = 0; tr < qr; ++tr) {
      const size_t row0 = qtiles.size();
      for (int tc = 0; tc < qc; ++tc) {
        const auto& l = per_tile[(size_t)tr * qc + tc];
        qtiles.push_back(make_int4((int)qlist.size(), (int)l.size(), tr * pmace::QT_R, tc * pmace::QT_C));
        qlist.insert(qlist.end(), l.begin(), l.end());
      }
      xcd_runs(qtiles, row0, qtiles.size());
    }
    if (qtiles.size() > split_tiles(p) || qlist.size() > split_list(p)) return PMACE_EDEVICE;
  }

  // Gather tables: per chunk, GT_R x GT_C tiles over the rows its patches
  // cover, each with the chunk's positions overlapping it in ascending order.
  const int chunk = chunk_of(p);
  const int nch = num_chunks(p);
  const int tiles_c = (n2 + pmace::GT_C - 1) / pmace::GT_C;
  std::vector<int4> tiles;
  std::vector<int> list;
  std::vector<int2> gitems, chunk_tiles(nch);
  {
    std::vector<std::vector<int>> per_tile;
    for (int g = 0; g < nch; ++g) {
      const int ja = g * chunk, jb = std::min(J, ja + chunk);
      int lo = n1, hi = 0;
      for (int j = ja; j < jb; ++j) {
        lo = std::min(lo, pos[2 * j]);
        hi = std::max(hi, pos[2 * j] + np);
      }
      const int tiles_r = (hi - lo + pmace::GT_R - 1) / pmace::GT_R;
      per_tile.assign((size_t)tiles_r * tiles_c, {});
      for (int j = ja; j < jb; ++j) {
        const int r = pos[2 * j] - lo, cc = pos[2 * j + 1];
        for (int tr = r / pmace::GT_R; tr <= (r + np - 1) / pmace::GT_R; ++tr)
          for (int tc = cc / pmace::GT_C; tc <= (cc + np - 1) / pmace::GT_C; ++tc)
            per_tile[(size_t)tr * tiles_c + tc].push_back(j);
      }
      chunk_tiles[g] = make_int2((int)gitems.size(), 0);
      size_t row0 = tiles.size();
      for (size_t t = 0; t < per_tile.size(); ++t) {
        if (t % tiles_c == 0) {
          if (np_large(np)) xcd_runs(tiles, row0, tiles.size());
          row0 = tiles.size();
        }
        if (per_tile[t].empty()) continue;
        const int tr = (int)(t / tiles_c), tc = (int)(t % tiles_c);
        gitems.push_back(make_int2(0, (int)tiles.size()));
        tiles.push_back(make_int4((int)list.size(), (int)per_tile[t].size(), lo + tr * pmace::GT_R,
                                  tc * pmace::GT_C));
        list.insert(list.end(), per_tile[t].begin(), per_tile[t].end());
      }
      if (np_large(np)) xcd_runs(tiles, row0, tiles.size());
      chunk_tiles[g].y = (int)gitems.size() - chunk_tiles[g].x;
    }
  }
  if (tiles.size() > max_tiles(p) || list.size() > max_list(p)) return PMACE_EDEVICE;

  // Row-spectrum states: per chunk, one item per object row its patches cover
  // and CR_W-wide segment of that row, listing the chunk's positions whose
  // patch covers the row and meets the segment, in ascending j.
  const bool rowspec = rowspec_allowed(p) && (sharp || !has_zero);
  std::vector<int4> citems, clist;
  std::vector<int2> chunk_rows(nch, make_int2(0, 0));
  if (rowspec) {
    const int nseg = cr_segments(p);
    const int rn = pmace::cr_round(np);
    std::vector<std::vector<int4>> per_row;
    for (int g = 0; g < nch; ++g) {
      const int ja = g * chunk, jb = std::min(J, ja + chunk);
      int lo = n1, hi = 0;
      for (int j = ja; j < jb; ++j) {
        lo = std::min(lo, pos[2 * j]);
        hi = std::max(hi, pos[2 * j] + np);
      }
      per_row.assign((size_t)(hi - lo) * nseg, {});
      for (int j = ja; j < jb; ++j) {
        const int r = pos[2 * j], cc = pos[2 * j + 1];
        for (int sg = cc / pmace::CR_W; sg <= (cc + np - 1) / pmace::CR_W; ++sg)
          for (int rr = 0; rr < np; ++rr)
            per_row[(size_t)(r + rr - lo) * nseg + sg].push_back(make_int4(j, rr, cc, 0));
      }
      chunk_rows[g] = make_int2((int)citems.size(), 0);
      for (size_t t = 0; t < per_row.size(); ++t) {
        if (per_row[t].empty()) continue;
        // By patch row, so that a round's rows share few weight rows (read
        // once into the cache), then each round by patch column, so the
        // entries covering a run of pixels are consecutive in it; ties in
        // ascending j.  The consensus sums each pixel in this order.
        auto& l = per_row[t];
        std::stable_sort(l.begin(), l.end(), [](const int4& a, const int4& b) { return a.y < b.y; });
        for (size_t r0 = 0; r0 < l.size(); r0 += (size_t)rn)
          std::stable_sort(l.begin() + r0, l.begin() + std::min(l.size(), r0 + (size_t)rn),
                           [](const int4& a, const int4& b) { return a.z < b.z; });
        citems.push_back(make_int4((int)clist.size(), (int)per_row[t].size(), lo + (int)(t / nseg),
                                   (int)(t % nseg) * pmace::CR_W));
        clist.insert(clist.end(), per_row[t].begin(), per_row[t].end());
      }
      chunk_rows[g].y = (int)citems.size() - chunk_rows[g].x;
    }
    if (citems.size() > cr_items(p) || clist.size() > cr_list(p)) return PMACE_EDEVICE;
  }
  std::vector<int2> items(J);
  for (int j = 0; j < J; ++j) items[j] = make_int2(0, j);
  const int nred = num_red(p);
  std::vector<int2> ritems(nred);
  for (int b = 0; b < nred; ++b) ritems[b] = make_int2(0, b);

  pmace_ctx* c = new (std::nothrow) pmace_ctx();
  if (!c) return PMACE_ENOMEM;
  c->prm = p;
  c->stream = st;
  c->sticky = PMACE_OK;
  c->graph_tried = false;
  c->resets = 0;
  if (hipGetDevice(&c->device) != hipSuccess) { delete c; return PMACE_EDEVICE; }

  const Layout L = layout_of(p);
  char* base = reinterpret_cast<char*>(align_up(reinterpret_cast<size_t>(workspace_d)));
  Recon& h = c->h;
  std::memset(&h, 0, sizeof(Recon));
  h.t = reinterpret_cast<float2*>(base + L.t);
  h.ys = reinterpret_cast<float*>(base + L.ys);
  h.pos = reinterpret_cast<int2*>(base + L.pos);
  h.d = reinterpret_cast<float2*>(base + L.d);
  h.pc = reinterpret_cast<float4*>(base + L.pc);
  h.gw = reinterpret_cast<float2*>(base + L.gw);
  h.omega64 = reinterpret_cast<double*>(base + L.omega64);
  h.dinv = reinterpret_cast<float2*>(base + L.dinv);
  h.laminv = reinterpret_cast<float*>(base + L.laminv);
  h.num = reinterpret_cast<float2*>(base + L.num);
  h.sold = reinterpret_cast<float2*>(base + L.sold);
  h.xbar = reinterpret_cast<float2*>(base + L.xbar);
  h.xhat = reinterpret_cast<float2*>(base + L.xhat);
  h.stage = reinterpret_cast<float2*>(base + L.stage);
  h.tiles = reinterpret_cast<int4*>(base + L.tiles);
  h.tile_list = reinterpret_cast<int*>(base + L.list);
  h.status = reinterpret_cast<unsigned*>(base + L.status);
  h.done = reinterpret_cast<int*>(base + L.status + 4);
  c->fitem = reinterpret_cast<int*>(base + L.status + 8);
  h.track = reinterpret_cast<double*>(base + L.status + 32);
  h.red = reinterpret_cast<double*>(base + L.red);
  h.twn = reinterpret_cast<float2*>(base + L.tw);
  h.fit = reinterpret_cast<double*>(base + L.fit);
  h.fit_bpp = split ? 4 : fit_bpp(p);
  h.split = split ? 1 : 0;
  h.dr = reinterpret_cast<float2*>(base + L.dr);
  h.part = h.stage;   // the split layout keeps its partial sums where the stage would be
  h.qtiles = reinterpret_cast<int4*>(base + L.qtiles);
  h.qlist = reinterpret_cast<int*>(base + L.qlist);
  h.qrows = split_rows(p);
  h.qcols = split_cols(p);
  h.nqt = (int)qtiles.size();
  h.rowspec = rowspec ? 1 : 0;
  h.citems = reinterpret_cast<int4*>(base + L.citems);
  h.clist = reinterpret_cast<int4*>(base + L.clist);
  h.xref = nullptr;
  h.mask = nullptr;
  h.n1 = n1;
  h.n2 = n2;
  h.np = np;
  h.np2f = (float)((double)np * np);
  h.J = J;
  h.method = p.method;
  if (sharp) {
    h.beta = p.beta;
    h.a = 0.f;
    h.two_rho = 2.f * p.beta;
    h.rho = 1.f;
    h.ka = (float)((1.0 - 2.0 * (double)p.beta) * inv_np2);
    h.yfac = 1.f;
  } else {
    h.beta = 0.f;
    h.a = p.alpha / (1.f + p.alpha);
    h.two_rho = 2.f * p.rho;
    h.rho = p.rho;
    h.ka = 0.f;
    h.yfac = (float)(1.0 + (double)p.alpha);
    const double rho = p.rho, a = (double)p.alpha / (1.0 + (double)p.alpha);
    h.sb = (float)((1.0 - 2.0 * rho * a) * inv_np2);
    h.s2r = (float)(2.0 * rho * inv_np2);
    h.has_zero = has_zero ? 1 : 0;
    h.cx = (float)(2.0 * (1.0 - rho));
    h.co = (float)((1.0 - rho) / rho);
    h.cn = (float)(1.0 / rho);
  }
  h.chunk = chunk;
  h.nt_stage = rowspec && (double)std::min(chunk, p.num_pos) * np * np * 8.0 > 512.0 * (1 << 20) ? 1 : 0;
  h.n_red = nred;
  h.ppw = p.ppw > 0 ? p.ppw : pmace::default_ppw(p.np);
  c->dev = reinterpret_cast<Recon*>(base + L.desc);
  c->items = reinterpret_cast<int2*>(base + L.items);
  c->gitems = reinterpret_cast<int2*>(base + L.gitems);
  c->ritems = reinterpret_cast<int2*>(base + L.ritems);
  c->ngitems = (int)gitems.size();
  c->chunk_tiles = chunk_tiles;
  c->chunk_rows = chunk_rows;

  const int zero = 0;
  std::vector<float> tw(512);
  for (int m = 0; m < np; ++m) {
    const double cv = std::cos(-2.0 * M_PI * m / np), sv = std::sin(-2.0 * M_PI * m / np);
    tw[2 * m] = std::fabs(cv) < 1e-15 ? 0.f : (float)cv;       // exact zeros at quarter turns
    tw[2 * m + 1] = std::fabs(sv) < 1e-15 ? 0.f : (float)sv;
  }
  auto fail = [&](pmace_status e) {
    pmace_destroy(c);
    return e;
  };
  if (hipMemcpyAsync(h.pos, pos.data(), (size_t)J * 8, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(h.d, probe.data(), np2 * 8, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(h.pc, pc.data(), np2 * 16, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(h.gw, gw.data(), np2 * 8, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(h.dinv, dinv.data(), np2 * 8, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(h.omega64, omega.data(), np2 * 8, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(h.tiles, tiles.data(), tiles.size() * 16, hipMemcpyHostToDevice, st) != hipSuccess ||
      (!list.empty() &&
       hipMemcpyAsync(h.tile_list, list.data(), list.size() * 4, hipMemcpyHostToDevice, st) != hipSuccess) ||
      hipMemcpyAsync(c->items, items.data(), items.size() * 8, hipMemcpyHostToDevice, st) != hipSuccess ||
      (!gitems.empty() &&
       hipMemcpyAsync(c->gitems, gitems.data(), gitems.size() * 8, hipMemcpyHostToDevice, st) != hipSuccess) ||
      hipMemcpyAsync(c->ritems, ritems.data(), ritems.size() * 8, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(c->fitem, &zero, 4, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(h.twn, tw.data(), (size_t)np * 8, hipMemcpyHostToDevice, st) != hipSuccess ||
      (split &&
       (hipMemcpyAsync(h.dr, dr.data(), dr.size() * 4, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(h.qtiles, qtiles.data(), qtiles.size() * 16, hipMemcpyHostToDevice, st) != hipSuccess ||
        (!qlist.empty() &&
         hipMemcpyAsync(h.qlist, qlist.data(), qlist.size() * 4, hipMemcpyHostToDevice, st) != hipSuccess))) ||
      (rowspec && !citems.empty() &&
       (hipMemcpyAsync(h.citems, citems.data(), citems.size() * 16, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(h.clist, clist.data(), clist.size() * 16, hipMemcpyHostToDevice, st) != hipSuccess)) ||
      hipMemsetAsync(h.status, 0, 4, st) != hipSuccess ||
      hipMemcpyAsync(c->dev, &c->h, sizeof(Recon), hipMemcpyHostToDevice, st) != hipSuccess)
    return fail(PMACE_EDEVICE);
  hipLaunchKernelGGL(reset_tracking_k, dim3(1), dim3(1), 0, st, h.done, h.track);
  const float yscale = (float)((double)np / (sharp ? 1.0 : 1.0 + (double)p.alpha));
  if (hipGetLastError() != hipSuccess ||
      pmace::launch_init(h, c->dev, intensity_d, yscale, (p.flags & PMACE_CENTERED_DC) ? 1 : 0,
                         reinterpret_cast<const float2*>(x0_d), c->chunk_tiles.data(), st) != hipSuccess)
    return fail(PMACE_EDEVICE);
  unsigned status = 0;
  if (hipMemcpyAsync(&status, h.status, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(PMACE_EDEVICE);
  if (status & 2u) return fail(PMACE_EINVAL);
  *out = c;
  return PMACE_OK;
}

pmace_status pmace_iterate(pmace_ctx* c, int32_t n_iter) {
  if (!c) return PMACE_ESTATE;
  if (n_iter < 0) return PMACE_EINVAL;
  if (n_iter == 0) return PMACE_OK;
  // a stop flag left by a batch would make the kernels skip this reconstruction
  if (hipMemsetAsync(c->h.done, 0, 4, c->stream) != hipSuccess) return record(c, PMACE_EDEVICE);
  ++c->resets;
  // One graph replays one iteration; a second replays kGraphIters of them in
  // a row, so long runs pay one launch per kGraphIters iterations.
  constexpr int kGraphIters = 32;
  if (!c->graph_tried && graphs_enabled()) {
    c->graph_tried = true;
    (void)capture(c->graph, [&](hipStream_t cs) { return enqueue_iteration(c, cs); });
    if (c->graph.x)
      (void)capture(c->graph_k, [&](hipStream_t cs) {
        for (int i = 0; i < kGraphIters; ++i) {
          const pmace_status s = enqueue_iteration(c, cs);
          if (s != PMACE_OK) return s;
        }
        return PMACE_OK;
      });
  }
  int k = 0;
  if (c->graph_k.x)
    for (; k + kGraphIters <= n_iter; k += kGraphIters)
      if (hipGraphLaunch(c->graph_k.x, c->stream) != hipSuccess) return record(c, PMACE_EDEVICE);
  for (; k < n_iter; ++k) {
    if (c->graph.x) {
      if (hipGraphLaunch(c->graph.x, c->stream) != hipSuccess) return record(c, PMACE_EDEVICE);
    } else {
      pmace_status s = enqueue_iteration(c, c->stream);
      if (s != PMACE_OK) return record(c, s);
    }
  }
  return PMACE_OK;
}

pmace_status pmace_reconstruct(pmace_ctx* c, void* xhat_d) {
  if (!c) return PMACE_ESTATE;
  if (!xhat_d) return PMACE_EINVAL;
  const size_t bytes = (size_t)c->prm.n1 * c->prm.n2 * 8;
  if (hipMemcpyAsync(xhat_d, c->h.xhat, bytes, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
    return record(c, PMACE_EDEVICE);
  return PMACE_OK;
}

pmace_status pmace_get_state(pmace_ctx* c, void* v_d) {
  if (!c) return PMACE_ESTATE;
  if (!v_d) return PMACE_EINVAL;
  if (pmace::launch_get_state(c->h, c->dev, reinterpret_cast<float2*>(v_d), c->stream) != hipSuccess)
    return record(c, PMACE_EDEVICE);
  return PMACE_OK;
}

pmace_status pmace_set_state(pmace_ctx* c, const void* v_d) {
  if (!c) return PMACE_ESTATE;
  if (!v_d) return PMACE_EINVAL;
  if (pmace::launch_set_state(c->h, c->dev, reinterpret_cast<const float2*>(v_d),
                              c->chunk_tiles.data(), c->stream) != hipSuccess)
    return record(c, PMACE_EDEVICE);
  return PMACE_OK;
}

pmace_status pmace_set_reference(pmace_ctx* c, const void* xref_d, const uint8_t* mask_d) {
  if (!c) return PMACE_ESTATE;
  c->h.xref = const_cast<float2*>(reinterpret_cast<const float2*>(xref_d));
  c->h.mask = xref_d ? const_cast<unsigned char*>(mask_d) : nullptr;
  if (hipMemcpyAsync(c->dev, &c->h, sizeof(Recon), hipMemcpyHostToDevice, c->stream) != hipSuccess)
    return record(c, PMACE_EDEVICE);
  // a batch reads its members through its own copies of their descriptors
  for (const auto& hb : c->holders)
    if (batch_recs_update(hb.first, hb.second, c->h, c->stream) != hipSuccess) return record(c, PMACE_EDEVICE);
  hipLaunchKernelGGL(reset_tracking_k, dim3(1), dim3(1), 0, c->stream, c->h.done, c->h.track);
  ++c->resets;
  if (hipGetLastError() != hipSuccess || hipStreamSynchronize(c->stream) != hipSuccess)
    return record(c, PMACE_EDEVICE);
  return PMACE_OK;
}

pmace_status pmace_nrmse(pmace_ctx* c, double* out) {
  if (!c) return PMACE_ESTATE;
  if (!out) return PMACE_EINVAL;
  if (!c->h.xref) return PMACE_ESTATE;
  if (pmace::launch_nrmse(c->dev, c->ritems, c->h.n_red, c->fitem, 1, 0, 0.f, 0, c->stream) !=
          hipSuccess ||
      hipMemcpyAsync(out, c->h.track + 1, 8, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return record(c, PMACE_EDEVICE);
  return PMACE_OK;
}

pmace_status pmace_set_stream(pmace_ctx* c, void* hip_stream) {
  if (!c) return PMACE_ESTATE;
  hipStream_t ns = reinterpret_cast<hipStream_t>(hip_stream);
  if (ns == c->stream) return PMACE_OK;
  // everything queued so far completes before the context's next work
  if (hipStreamSynchronize(c->stream) != hipSuccess) return record(c, PMACE_EDEVICE);
  c->stream = ns;
  return PMACE_OK;
}

pmace_status pmace_data_fit(pmace_ctx* c, double* out) {
  if (!c) return PMACE_ESTATE;
  if (!out) return PMACE_EINVAL;
  if (pmace::launch_fit_member(c->h, c->dev, 0, c->stream) != hipSuccess ||
      pmace::launch_fit_finish(c->dev, c->fitem, 1, 0, 0.f, 0, c->stream) != hipSuccess ||
      hipMemcpyAsync(out, c->h.track + 6, 8, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return record(c, PMACE_EDEVICE);
  return PMACE_OK;
}

pmace_status pmace_sync(pmace_ctx* c) {
  if (!c) return PMACE_ESTATE;
  unsigned status = 0;
  if (hipMemcpyAsync(&status, c->h.status, 4, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return record(c, PMACE_EDEVICE);
  if (c->sticky != PMACE_OK) return c->sticky;
  if (status & 1u) return record(c, PMACE_EDIVERGED);
  return PMACE_OK;
}

int32_t pmace_agent_kind(const pmace_ctx* c) {
  if (!c) return -1;
  if (c->h.split) return PMACE_AGENT_SPLIT;
  if (c->h.rowspec) return PMACE_AGENT_ROWSPEC;
  return np_large(c->prm.np) ? PMACE_AGENT_THREE_PASS : PMACE_AGENT_WHOLE_PATCH;
}

void pmace_destroy(pmace_ctx* c) {
  if (!c) return;
  // a batch still holding this context (a caller error) must not reach it
  for (const auto& hb : c->holders) batch_forget(hb.first, hb.second);
  (void)hipStreamSynchronize(c->stream);
  c->graph.release();
  c->graph_k.release();
  delete c;
}

pmace_status pmace_fft2(int32_t np, int32_t count, const void* in_d, void* out_d, int32_t inverse,
                        void* hip_stream) {
  if (count < 0 || !in_d || !out_d) return PMACE_EINVAL;
  if (!np_supported(np)) return np < 1 ? PMACE_EINVAL : PMACE_EUNSUPPORTED;
  if (count == 0) return PMACE_OK;
  hipError_t e = pmace::launch_fft2(np, count, reinterpret_cast<const float2*>(in_d),
                                    reinterpret_cast<float2*>(out_d), inverse ? 1 : 0,
                                    reinterpret_cast<hipStream_t>(hip_stream));
  return e == hipSuccess ? PMACE_OK : PMACE_EDEVICE;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Batches
// ---------------------------------------------------------------------------
namespace {

int class_of(int np) {
  for (int k = 0; k < kClasses; ++k)
    if (np == kSmallNp[k]) return k;
  return -1;
}

struct BatchLayout {
  size_t recs, items[kClasses], gitems[kClasses], ritems, fitems, total;
  int nitems[kClasses], ngitems[kClasses], nritems;
};

BatchLayout batch_layout(pmace_ctx* const* ctxs, int n) {
  BatchLayout L{};
  for (int i = 0; i < n; ++i) {
    const int k = own_chain(ctxs[i]) ? -1 : class_of(ctxs[i]->prm.np);
    if (k >= 0) {
      L.nitems[k] += ctxs[i]->prm.num_pos;
      L.ngitems[k] += ctxs[i]->ngitems;
    }
    L.nritems += ctxs[i]->h.n_red;
  }
  size_t o = 0;
  L.recs = o;    o = align_up(o + (size_t)n * sizeof(Recon));
  for (int k = 0; k < kClasses; ++k) {
    L.items[k] = o;  o = align_up(o + (size_t)L.nitems[k] * 8);
    L.gitems[k] = o; o = align_up(o + (size_t)L.ngitems[k] * 8);
  }
  L.ritems = o;  o = align_up(o + (size_t)L.nritems * 8);
  L.fitems = o;  o = align_up(o + (size_t)n * 4);
  L.total = o;
  return L;
}

pmace_status check_members(pmace_ctx* const* ctxs, int32_t n) {
  if (!ctxs || n < 1) return PMACE_EINVAL;
  for (int i = 0; i < n; ++i) {
    if (!ctxs[i]) return PMACE_ESTATE;
    if (ctxs[i]->prm.method != PMACE_METHOD_PMACE) return PMACE_EUNSUPPORTED;
    if (ctxs[i]->stream != ctxs[0]->stream || ctxs[i]->device != ctxs[0]->device) return PMACE_EINVAL;
    for (int k = 0; k < i; ++k)
      if (ctxs[k] == ctxs[i]) return PMACE_EINVAL;
  }
  return PMACE_OK;
}

pmace_status enqueue_batch_iteration(pmace_batch* b, hipStream_t st, bool lanes, bool check) {
  // Np > 128 members are independent chains of kernels spread over the lanes;
  // they fork before the merged launches of the smaller members, so both run
  // at once (the small ones are latency-bound and leave most CUs free)
  bool any_large = false;
  for (int i = 0; i < b->n; ++i) any_large = any_large || (own_chain(b->ctxs[i]) && !b->pruned[i]);
  const bool forked = lanes && any_large;
  if (forked) {
    PM_HIP(hipEventRecord(b->fork, st));
    for (int l = 0; l < 4; ++l) PM_HIP(hipStreamWaitEvent(b->lanes[l], b->fork, 0));
  }
  for (int k = 0; k < kClasses; ++k)
    if (b->nitems[k] > 0)
      PM_HIP(pmace::launch_small_batch(kSmallNp[k], b->recs, b->items[k], b->nitems[k], b->gitems[k],
                                       b->ngitems[k], b->ppw[k], st));
  int lane = 0;
  for (int i = 0; i < b->n; ++i) {
    pmace_ctx* c = b->ctxs[i];
    if (!own_chain(c) || b->pruned[i]) continue;
    hipStream_t ls = st;
    if (forked) {
      ls = b->lanes[lane];
      lane = (lane + 1) % 4;
    }
    if (c->h.split)
      PM_HIP(pmace::launch_split_iteration(c->h, 1, ls));
    else
      PM_HIP(pmace::launch_large_iteration(c->h, b->recs + i, c->chunk_tiles.data(), c->chunk_rows.data(), ls));
  }
  if (forked)
    for (int l = 0; l < 4; ++l) {
      PM_HIP(hipEventRecord(b->join[l], b->lanes[l]));
      PM_HIP(hipStreamWaitEvent(st, b->join[l], 0));
    }
  PM_HIP(pmace::launch_tick(b->recs, b->fitems, b->n, b->rule.max_iter, 0, st));
  if (check && b->rule.criterion == PMACE_STOP_NRMSE) {
    PM_HIP(pmace::launch_nrmse(b->recs, b->ritems, b->nritems, b->fitems, b->n, 1, b->rule.tol,
                               b->rule.min_iter, st));
  } else if (check) {
    for (int k = 0; k < kClasses; ++k)
      PM_HIP(pmace::launch_fit_batch(kSmallNp[k], b->recs, b->items[k], b->nitems[k], st));
    for (int i = 0; i < b->n; ++i)
      if (own_chain(b->ctxs[i]) && !b->pruned[i])
        PM_HIP(pmace::launch_fit_member(b->ctxs[i]->h, b->recs + i, 1, st));
    PM_HIP(pmace::launch_fit_finish(b->recs, b->fitems, b->n, 1, b->rule.tol, b->rule.min_iter, st));
  }
  PM_HIP(pmace::launch_tick(b->recs, b->fitems, b->n, b->rule.max_iter, 1, st));
  return PMACE_OK;
}

// The launches of the batch changed: the captured graphs are destroyed once
// the launches of them in flight have finished, and captured again on the next
// step.
pmace_status drop_graphs(pmace_batch* b) {
  if (hipStreamSynchronize(b->stream) != hipSuccess) return PMACE_EDEVICE;
  b->graph.release();
  b->graph_check.release();
  b->graph_tried = false;
  return PMACE_OK;
}

hipError_t batch_recs_update(pmace_batch* b, int i, const Recon& h, hipStream_t st) {
  return hipMemcpyAsync(b->recs + i, &h, sizeof(Recon), hipMemcpyHostToDevice, st);
}

void batch_forget(pmace_batch* b, int i) { b->ctxs[i] = nullptr; }

void batch_release(pmace_batch* b) {
  for (pmace_ctx* c : b->ctxs) {
    if (!c) continue;
    auto& hs = c->holders;
    for (size_t k = 0; k < hs.size();)
      if (hs[k].first == b) hs.erase(hs.begin() + (long)k);
      else ++k;
  }
  b->graph.release();
  b->graph_check.release();
  for (int l = 0; l < 4; ++l) {
    if (b->lanes[l]) (void)hipStreamDestroy(b->lanes[l]);
    if (b->join[l]) (void)hipEventDestroy(b->join[l]);
  }
  if (b->fork) (void)hipEventDestroy(b->fork);
  delete b;
}

}  // namespace

extern "C" {

size_t pmace_batch_footprint(pmace_ctx* const* ctxs, int32_t n) {
  if (check_members(ctxs, n) != PMACE_OK) return 0;
  return batch_layout(ctxs, n).total + kAlign;
}

pmace_status pmace_batch_create(pmace_ctx* const* ctxs, int32_t n, const pmace_stop_rule* rule,
                                void* workspace_d, size_t ws_bytes, pmace_batch** out) {
  if (!out) return PMACE_EINVAL;
  *out = nullptr;
  pmace_status ps = check_members(ctxs, n);
  if (ps != PMACE_OK) return ps;
  if (!rule || !workspace_d || rule->min_iter < 0 || rule->max_iter < 1 || !std::isfinite(rule->tol) ||
      (rule->criterion != PMACE_STOP_NRMSE && rule->criterion != PMACE_STOP_DATA_FIT) ||
      rule->check_every < 0)
    return PMACE_EINVAL;
  const BatchLayout L = batch_layout(ctxs, n);
  if (ws_bytes < L.total + kAlign) return PMACE_ENOMEM;
  pmace_batch* b = new (std::nothrow) pmace_batch();
  if (!b) return PMACE_ENOMEM;
  b->n = n;
  b->stream = ctxs[0]->stream;
  b->ctxs.assign(ctxs, ctxs + n);
  b->rule = *rule;
  if (b->rule.check_every == 0) b->rule.check_every = 1;
  b->graph_tried = false;
  b->iters = 0;
  b->step_calls = 0;
  b->pruned.assign(n, 0);
  b->pruned_at.assign(n, 0);
  char* base = reinterpret_cast<char*>(align_up(reinterpret_cast<size_t>(workspace_d)));
  b->recs = reinterpret_cast<Recon*>(base + L.recs);
  std::vector<Recon> recs(n);
  std::vector<int2> items[kClasses], gitems[kClasses], ritems;
  std::vector<int> fitems(n);
  for (int i = 0; i < n; ++i) {
    pmace_ctx* c = ctxs[i];
    recs[i] = c->h;
    fitems[i] = i;
    for (int r = 0; r < c->h.n_red; ++r) ritems.push_back(make_int2(i, r));
    const int k = own_chain(c) ? -1 : class_of(c->prm.np);
    if (k < 0) continue;
    if (items[k].empty()) b->ppw[k] = c->h.ppw;   // the class takes its first member's choice
    for (int j = 0; j < c->prm.num_pos; ++j) items[k].push_back(make_int2(i, j));
    for (int t = 0; t < c->ngitems; ++t) gitems[k].push_back(make_int2(i, t));
  }
  for (int l = 0; l < 4; ++l) {
    if (hipStreamCreateWithFlags(&b->lanes[l], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->join[l], hipEventDisableTiming) != hipSuccess) {
      batch_release(b);
      return PMACE_EDEVICE;
    }
  }
  if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess) {
    batch_release(b);
    return PMACE_EDEVICE;
  }
  hipStream_t st = b->stream;
  bool ok = hipMemcpyAsync(b->recs, recs.data(), (size_t)n * sizeof(Recon), hipMemcpyHostToDevice,
                           st) == hipSuccess;
  for (int k = 0; k < kClasses; ++k) {
    b->items[k] = reinterpret_cast<int2*>(base + L.items[k]);
    b->gitems[k] = reinterpret_cast<int2*>(base + L.gitems[k]);
    b->nitems[k] = (int)items[k].size();
    b->ngitems[k] = (int)gitems[k].size();
    if (!items[k].empty())
      ok = ok && hipMemcpyAsync(b->items[k], items[k].data(), items[k].size() * 8,
                                hipMemcpyHostToDevice, st) == hipSuccess;
    if (!gitems[k].empty())
      ok = ok && hipMemcpyAsync(b->gitems[k], gitems[k].data(), gitems[k].size() * 8,
                                hipMemcpyHostToDevice, st) == hipSuccess;
  }
  b->ritems = reinterpret_cast<int2*>(base + L.ritems);
  b->nritems = (int)ritems.size();
  b->fitems = reinterpret_cast<int*>(base + L.fitems);
  ok = ok && hipMemcpyAsync(b->ritems, ritems.data(), ritems.size() * 8, hipMemcpyHostToDevice, st) ==
                 hipSuccess;
  ok = ok && hipMemcpyAsync(b->fitems, fitems.data(), (size_t)n * 4, hipMemcpyHostToDevice, st) ==
                 hipSuccess;
  ok = ok && hipStreamSynchronize(st) == hipSuccess;
  if (!ok) {
    batch_release(b);
    return PMACE_EDEVICE;
  }
  for (int i = 0; i < n; ++i) ctxs[i]->holders.emplace_back(b, i);
  *out = b;
  return PMACE_OK;
}

pmace_status pmace_batch_step(pmace_batch* b, int32_t n_iter) {
  if (!b) return PMACE_ESTATE;
  if (n_iter < 0) return PMACE_EINVAL;
  const int every = b->rule.check_every;
  // a pruned member whose stop flag the host has cleared runs again
  bool changed = false;
  for (int i = 0; i < b->n; ++i)
    if (b->pruned[i] && b->ctxs[i]->resets != b->pruned_at[i]) {
      b->pruned[i] = 0;
      changed = true;
    }
  if (changed && drop_graphs(b) != PMACE_OK) return PMACE_EDEVICE;
  // A batch whose membership changes often (a serving loop rebuilds it on
  // every admission and retirement) would spend more host time capturing and
  // instantiating graphs than it saves, so the first kCaptureAfter calls
  // launch eagerly and only a batch that lives longer is captured.
  constexpr int kCaptureAfter = 2;
  if (!b->graph_tried && graphs_enabled() && b->step_calls >= kCaptureAfter) {
    b->graph_tried = true;
    (void)capture(b->graph_check,
                  [&](hipStream_t cs) { return enqueue_batch_iteration(b, cs, true, true); });
    if (every > 1)
      (void)capture(b->graph, [&](hipStream_t cs) { return enqueue_batch_iteration(b, cs, true, false); });
  }
  for (int k = 0; k < n_iter; ++k) {
    // the stop rule is evaluated after every `every`-th iteration of the batch
    const bool check = (b->iters + 1) % every == 0;
    ++b->iters;
    const Graph& g = check ? b->graph_check : b->graph;
    if (g.x) {
      if (hipGraphLaunch(g.x, b->stream) != hipSuccess) return PMACE_EDEVICE;
    } else {
      pmace_status s = enqueue_batch_iteration(b, b->stream, true, check);
      if (s != PMACE_OK) return s;
    }
  }
  ++b->step_calls;
  return PMACE_OK;
}

pmace_status pmace_batch_poll_fit(pmace_batch* b, int32_t* done, double* nrmse, int32_t* iters,
                                  double* data_fit) {
  if (!b) return PMACE_ESTATE;
  std::vector<int> dn(b->n);
  std::vector<double> tr(8 * (size_t)b->n);
  for (int i = 0; i < b->n; ++i) {
    if (hipMemcpyAsync(&dn[i], b->ctxs[i]->h.done, 4, hipMemcpyDeviceToHost, b->stream) != hipSuccess ||
        hipMemcpyAsync(&tr[8 * i], b->ctxs[i]->h.track, 64, hipMemcpyDeviceToHost, b->stream) != hipSuccess)
      return PMACE_EDEVICE;
  }
  if (hipStreamSynchronize(b->stream) != hipSuccess) return PMACE_EDEVICE;
  bool changed = false;
  for (int i = 0; i < b->n; ++i)
    if (dn[i] && own_chain(b->ctxs[i]) && !b->pruned[i]) {
      b->pruned[i] = 1;
      b->pruned_at[i] = b->ctxs[i]->resets;
      changed = true;
    }
  if (changed && drop_graphs(b) != PMACE_OK) return PMACE_EDEVICE;
  for (int i = 0; i < b->n; ++i) {
    if (done) done[i] = dn[i];
    if (nrmse) nrmse[i] = tr[8 * i + 1];
    if (iters) iters[i] = (int32_t)tr[8 * i + 3];
    if (data_fit) data_fit[i] = tr[8 * i + 4];
  }
  return PMACE_OK;
}

pmace_status pmace_batch_poll(pmace_batch* b, int32_t* done, double* nrmse, int32_t* iters) {
  return pmace_batch_poll_fit(b, done, nrmse, iters, nullptr);
}

void pmace_batch_destroy(pmace_batch* b) {
  if (!b) return;
  (void)hipStreamSynchronize(b->stream);
  batch_release(b);
}

}  // extern "C"
