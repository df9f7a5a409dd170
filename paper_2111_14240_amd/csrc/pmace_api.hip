// C ABI of libpmace.so (declared in include/pmace.h).
//
// Host responsibilities: argument validation, the workspace layout, the FP64
// tables computed once per reconstruction (|d|^kappa, d^{-1}, Lambda^{-1} of
// eq. (11)), and replaying one captured iteration as a HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "pmace.h"
#include "pmace_internal.hpp"

using pmace::DevState;

struct pmace_ctx {
  pmace_params prm;
  hipStream_t stream;
  int device;
  DevState s;
  // one iteration captured as a graph and replayed on `stream`
  hipStream_t cap_stream;
  hipGraph_t graph;
  hipGraphExec_t exec;
  bool graph_ready;
  bool use_graph;
  pmace_status sticky;  // first asynchronous failure seen
  std::vector<int4> chunk_info;  // per chunk: (first tile, tiles, first tile row, tiles per row)
};

namespace {

constexpr size_t kAlign = 256;

inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

bool np_supported(int np) { return np == 32 || np == 64 || np == 128 || np == 256; }

// Positions per chunk: Np <= 128 runs all positions in one fused launch;
// Np = 256 stages chunk*Np^2 spectra between its three passes.
int chunk_of(const pmace_params& p) {
  int c = p.num_pos;
  if (p.np == 256 && p.chunk > 0) c = p.chunk;
  else if (p.np == 256) c = 128;
  if (c > p.num_pos) c = p.num_pos;
  return c;
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

pmace_status check_params(const pmace_params* p) {
  if (!p) return PMACE_EINVAL;
  if (p->np < 1 || p->num_pos < 1 || p->n1 < p->np || p->n2 < p->np) return PMACE_EINVAL;
  if (!(std::isfinite(p->alpha) && p->alpha >= 0.f)) return PMACE_EINVAL;
  if (!(std::isfinite(p->kappa) && p->kappa >= 0.f)) return PMACE_EINVAL;
  if (!(std::isfinite(p->rho) && p->rho > 0.f && p->rho < 1.f)) return PMACE_EINVAL;
  if (p->flags & ~PMACE_CENTERED_DC) return PMACE_EINVAL;
  if (p->chunk < 0) return PMACE_EINVAL;
  if ((long long)p->n1 * p->n2 > (1LL << 30)) return PMACE_EINVAL;
  if (!np_supported(p->np)) return PMACE_EUNSUPPORTED;
  return PMACE_OK;
}

// Section offsets inside the workspace (relative to the aligned base).
struct Layout {
  size_t t, ys, pos, d, pc, laminv, num, xbar, xhat, status, stage, tiles, list, total;
};

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
  L.laminv = o;  o = align_up(o + npx * 4);
  L.num = o;     o = align_up(o + npx * 8);
  L.xbar = o;    o = align_up(o + npx * 8);
  L.xhat = o;    o = align_up(o + npx * 8);
  L.status = o;  o = align_up(o + 16);
  L.stage = o;   o = align_up(o + (size_t)chunk_of(p) * np2 * 8);
  L.tiles = o;   o = align_up(o + max_tiles(p) * 8);
  L.list = o;    o = align_up(o + max_list(p) * 4);
  L.total = o;
  return L;
}

#define PM_HIP(call)                                   \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return PMACE_EDEVICE;        \
  } while (0)

pmace_status record(pmace_ctx* c, pmace_status s) {
  if (s != PMACE_OK && c->sticky == PMACE_OK) c->sticky = s;
  return s;
}

pmace_status enqueue_iteration(pmace_ctx* c, hipStream_t st) {
  PM_HIP(pmace::launch_agent(c->s, st));
  return PMACE_OK;
}

pmace_status build_graph(pmace_ctx* c) {
  PM_HIP(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
  PM_HIP(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
  pmace_status s = enqueue_iteration(c, c->cap_stream);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
  if (s != PMACE_OK) return s;
  if (e != hipSuccess || !g) return PMACE_EDEVICE;
  c->graph = g;
  PM_HIP(hipGraphInstantiate(&c->exec, g, nullptr, nullptr, 0));
  c->graph_ready = true;
  return PMACE_OK;
}

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
  std::vector<float> pc(4 * np2);
  std::vector<double> omega(np2);
  const double inv_np2 = 1.0 / ((double)np * np);
  for (size_t i = 0; i < np2; ++i) {
    const std::complex<double> dd(probe[i].real(), probe[i].imag());
    const double mag = std::abs(dd);
    omega[i] = std::pow(mag, (double)p.kappa);
    if (mag == 0.0) omega[i] = (p.kappa == 0.f) ? 1.0 : 0.0;
    std::complex<double> di(0.0, 0.0);
    if (mag != 0.0) di = inv_np2 / dd;
    pc[4 * i + 0] = (float)di.real();
    pc[4 * i + 1] = (float)di.imag();
    pc[4 * i + 2] = (float)omega[i];
    pc[4 * i + 3] = mag == 0.0 ? 1.f : 0.f;
  }
  std::vector<double> lam(npx, 0.0);
  for (int j = 0; j < J; ++j) {
    const int r0 = pos[2 * j], c0 = pos[2 * j + 1];
    for (int r = 0; r < np; ++r) {
      double* lr = &lam[(size_t)(r0 + r) * n2 + c0];
      const double* orow = &omega[(size_t)r * np];
      for (int c = 0; c < np; ++c) lr[c] += orow[c];
    }
  }
  std::vector<float> laminv(npx);
  for (size_t i = 0; i < npx; ++i) laminv[i] = lam[i] != 0.0 ? (float)(1.0 / lam[i]) : 0.f;

  pmace_ctx* c = new (std::nothrow) pmace_ctx();
  if (!c) return PMACE_ENOMEM;
  c->prm = p;
  c->stream = st;
  c->sticky = PMACE_OK;
  c->graph_ready = false;
  c->cap_stream = nullptr;
  c->graph = nullptr;
  c->exec = nullptr;
  {
    const char* e = std::getenv("PMACE_NO_GRAPH");
    c->use_graph = !(e && e[0] == '1');
  }
  if (hipGetDevice(&c->device) != hipSuccess) { delete c; return PMACE_EDEVICE; }

  const Layout L = layout_of(p);
  char* base = reinterpret_cast<char*>(align_up(reinterpret_cast<size_t>(workspace_d)));
  DevState& s = c->s;
  s.t = reinterpret_cast<float2*>(base + L.t);
  s.ys = reinterpret_cast<float*>(base + L.ys);
  s.pos = reinterpret_cast<int2*>(base + L.pos);
  s.d = reinterpret_cast<float2*>(base + L.d);
  s.pc = reinterpret_cast<float4*>(base + L.pc);
  s.laminv = reinterpret_cast<float*>(base + L.laminv);
  s.num = reinterpret_cast<float*>(base + L.num);
  s.xbar = reinterpret_cast<float2*>(base + L.xbar);
  s.xhat = reinterpret_cast<float2*>(base + L.xhat);
  s.status = reinterpret_cast<unsigned*>(base + L.status);
  s.stage = reinterpret_cast<float2*>(base + L.stage);
  s.tiles = reinterpret_cast<int2*>(base + L.tiles);
  s.tile_list = reinterpret_cast<int*>(base + L.list);
  s.n1 = n1;
  s.n2 = n2;
  s.np = np;
  s.J = J;
  s.a = p.alpha / (1.f + p.alpha);
  s.rho = p.rho;
  s.chunk = chunk_of(p);
  // Gather tables: per chunk, GT_R x GT_C tiles over the rows its patches
  // cover, each with the chunk's positions overlapping it in ascending order.
  std::vector<int2> tiles;
  std::vector<int> list;
  {
    const int nch = num_chunks(p);
    const int tiles_c = (n2 + pmace::GT_C - 1) / pmace::GT_C;
    c->chunk_info.resize(nch);
    std::vector<std::vector<int>> per_tile;
    for (int g = 0; g < nch; ++g) {
      const int ja = g * s.chunk, jb = std::min(J, ja + s.chunk);
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
      c->chunk_info[g] = make_int4((int)tiles.size(), (int)per_tile.size(), lo, tiles_c);
      for (auto& v : per_tile) {
        tiles.push_back(make_int2((int)list.size(), (int)v.size()));
        list.insert(list.end(), v.begin(), v.end());
      }
    }
  }
  if (tiles.size() > max_tiles(p) || list.size() > max_list(p)) { delete c; return PMACE_EDEVICE; }
  s.chunk_info = c->chunk_info.data();

  auto fail = [&](pmace_status e) { delete c; return e; };
  if (hipMemcpyAsync(s.pos, pos.data(), (size_t)J * 8, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(s.d, probe.data(), np2 * 8, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(s.pc, pc.data(), np2 * 16, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(s.laminv, laminv.data(), npx * 4, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(s.tiles, tiles.data(), tiles.size() * 8, hipMemcpyHostToDevice, st) != hipSuccess ||
      (!list.empty() &&
       hipMemcpyAsync(s.tile_list, list.data(), list.size() * 4, hipMemcpyHostToDevice, st) != hipSuccess) ||
      hipMemsetAsync(s.status, 0, 16, st) != hipSuccess)
    return fail(PMACE_EDEVICE);
  const float yscale = (float)((double)np / (1.0 + (double)p.alpha));
  if (pmace::launch_init_amplitudes(s, intensity_d, yscale, (p.flags & PMACE_CENTERED_DC) ? 1 : 0,
                                    st) != hipSuccess ||
      pmace::launch_init_state(s, reinterpret_cast<const float2*>(x0_d), st) != hipSuccess)
    return fail(PMACE_EDEVICE);
  unsigned status = 0;
  if (hipMemcpyAsync(&status, s.status, 4, hipMemcpyDeviceToHost, st) != hipSuccess ||
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
  if (c->use_graph) {
    if (!c->graph_ready) {
      pmace_status s = build_graph(c);
      if (s != PMACE_OK) {
        c->use_graph = false;  // fall back to direct launches of the same kernels
      }
    }
  }
  for (int k = 0; k < n_iter; ++k) {
    if (c->use_graph && c->graph_ready) {
      if (hipGraphLaunch(c->exec, c->stream) != hipSuccess) return record(c, PMACE_EDEVICE);
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
  if (hipMemcpyAsync(xhat_d, c->s.xhat, bytes, hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
    return record(c, PMACE_EDEVICE);
  return PMACE_OK;
}

pmace_status pmace_get_state(pmace_ctx* c, void* v_d) {
  if (!c) return PMACE_ESTATE;
  if (!v_d) return PMACE_EINVAL;
  if (pmace::launch_get_state(c->s, reinterpret_cast<float2*>(v_d), c->stream) != hipSuccess)
    return record(c, PMACE_EDEVICE);
  return PMACE_OK;
}

pmace_status pmace_set_state(pmace_ctx* c, const void* v_d) {
  if (!c) return PMACE_ESTATE;
  if (!v_d) return PMACE_EINVAL;
  if (pmace::launch_set_state(c->s, reinterpret_cast<const float2*>(v_d), c->stream) != hipSuccess)
    return record(c, PMACE_EDEVICE);
  return PMACE_OK;
}

pmace_status pmace_sync(pmace_ctx* c) {
  if (!c) return PMACE_ESTATE;
  unsigned status = 0;
  if (hipMemcpyAsync(&status, c->s.status, 4, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
      hipStreamSynchronize(c->stream) != hipSuccess)
    return record(c, PMACE_EDEVICE);
  if (c->sticky != PMACE_OK) return c->sticky;
  if (status & 1u) return record(c, PMACE_EDIVERGED);
  return PMACE_OK;
}

void pmace_destroy(pmace_ctx* c) {
  if (!c) return;
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  if (c->exec) (void)hipGraphExecDestroy(c->exec);
  if (c->graph) (void)hipGraphDestroy(c->graph);
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
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
