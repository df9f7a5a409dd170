// A PMACE reconstruction driven from C++ through the C ABI alone (no Python,
// no PyTorch): a synthetic object and probe are made on the host, the
// measurements are simulated on the device (eq. (1), eq. (16)), and the
// reconstruction is iterated with the data-fit cost of eq. (4) reported as it
// goes.  Prints one line per report and a final JSON line.
//
//   pmace_demo [n] [np] [scan] [step] [peak] [iterations]
//   defaults:   512  128  15     24     1e5    100
#include <hip/hip_runtime_api.h>

#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "pmace.h"

namespace {

#define CHECK_HIP(x)                                                              \
  do {                                                                            \
    hipError_t e_ = (x);                                                          \
    if (e_ != hipSuccess) {                                                       \
      std::fprintf(stderr, "%s:%d %s\n", __FILE__, __LINE__, hipGetErrorString(e_)); \
      std::exit(2);                                                               \
    }                                                                             \
  } while (0)

#define CHECK_PM(x)                                                                   \
  do {                                                                                \
    pmace_status s_ = (x);                                                            \
    if (s_ != PMACE_OK) {                                                             \
      std::fprintf(stderr, "%s:%d %s\n", __FILE__, __LINE__, pmace_status_str(s_));   \
      std::exit(3);                                                                   \
    }                                                                                 \
  } while (0)

using cf = std::complex<float>;

}  // namespace

int main(int argc, char** argv) {
  const int n = argc > 1 ? std::atoi(argv[1]) : 512;
  const int np = argc > 2 ? std::atoi(argv[2]) : 128;
  const int scan = argc > 3 ? std::atoi(argv[3]) : 15;
  const int step = argc > 4 ? std::atoi(argv[4]) : 24;
  const double peak = argc > 5 ? std::atof(argv[5]) : 1e5;
  const int iters = argc > 6 ? std::atoi(argv[6]) : 100;
  const int J = scan * scan;
  if ((scan - 1) * step + np > n) {
    std::fprintf(stderr, "the raster does not fit the object\n");
    return 1;
  }

  // Object: smooth magnitude in [0.5, 1] and phase in [-pi/2, pi/2].
  std::vector<cf> x((size_t)n * n);
  for (int r = 0; r < n; ++r)
    for (int c = 0; c < n; ++c) {
      const double a = 0.75 + 0.25 * std::sin(0.031 * r) * std::cos(0.027 * c);
      const double ph = 0.5 * M_PI * std::sin(0.019 * r + 0.023 * c);
      x[(size_t)r * n + c] = cf((float)(a * std::cos(ph)), (float)(a * std::sin(ph)));
    }
  // Probe: Gaussian (sigma = np/4) with a quadratic phase.
  std::vector<cf> d((size_t)np * np);
  for (int r = 0; r < np; ++r)
    for (int c = 0; c < np; ++c) {
      const double yy = r - np / 2.0 + 0.5, xx = c - np / 2.0 + 0.5, s = np / 4.0;
      const double rr = (yy * yy + xx * xx) / (s * s);
      const double ph = M_PI * 4.0 * (yy * yy + xx * xx) / ((double)np * np);
      const double m = std::exp(-0.5 * rr);
      d[(size_t)r * np + c] = cf((float)(m * std::cos(ph)), (float)(m * std::sin(ph)));
    }
  // Centred raster.
  std::vector<int32_t> pos(2 * (size_t)J);
  const int off = (n - ((scan - 1) * step + np)) / 2;
  for (int i = 0; i < scan; ++i)
    for (int k = 0; k < scan; ++k) {
      pos[2 * (i * scan + k)] = off + i * step;
      pos[2 * (i * scan + k) + 1] = off + k * step;
    }

  hipStream_t st;
  CHECK_HIP(hipStreamCreate(&st));
  void *x_d, *d_d, *pos_d, *z_d, *sim_ws, *ws, *xh_d;
  CHECK_HIP(hipMalloc(&x_d, x.size() * sizeof(cf)));
  CHECK_HIP(hipMalloc(&d_d, d.size() * sizeof(cf)));
  CHECK_HIP(hipMalloc(&pos_d, pos.size() * sizeof(int32_t)));
  CHECK_HIP(hipMalloc(&z_d, (size_t)J * np * np * sizeof(float)));
  CHECK_HIP(hipMalloc(&xh_d, x.size() * sizeof(cf)));
  CHECK_HIP(hipMemcpy(x_d, x.data(), x.size() * sizeof(cf), hipMemcpyHostToDevice));
  CHECK_HIP(hipMemcpy(d_d, d.data(), d.size() * sizeof(cf), hipMemcpyHostToDevice));
  CHECK_HIP(hipMemcpy(pos_d, pos.data(), pos.size() * sizeof(int32_t), hipMemcpyHostToDevice));

  // Measurements on the device; the photon scaling goes into the probe.
  const size_t sim_bytes = pmace_simulate_footprint(np, J);
  CHECK_HIP(hipMalloc(&sim_ws, sim_bytes));
  double scale = 1.0;
  CHECK_PM(pmace_simulate(n, n, np, J, d_d, static_cast<const int32_t*>(pos_d), x_d, peak, 1234,
                          static_cast<float*>(z_d), sim_ws, sim_bytes, &scale, st));
  for (auto& v : d) v *= (float)std::sqrt(scale);
  CHECK_HIP(hipMemcpy(d_d, d.data(), d.size() * sizeof(cf), hipMemcpyHostToDevice));

  pmace_params p{};
  p.n1 = n;
  p.n2 = n;
  p.np = np;
  p.num_pos = J;
  p.alpha = 0.5f;
  p.kappa = 1.25f;
  p.rho = 0.5f;
  p.method = PMACE_METHOD_PMACE;
  const size_t fp = pmace_footprint(&p);
  if (fp == 0) {
    std::fprintf(stderr, "unsupported parameters\n");
    return 1;
  }
  CHECK_HIP(hipMalloc(&ws, fp));
  pmace_ctx* ctx = nullptr;
  CHECK_PM(pmace_init(&p, d_d, static_cast<const int32_t*>(pos_d), static_cast<const float*>(z_d),
                      nullptr, ws, fp, st, &ctx));

  double cost = 0.0;
  CHECK_PM(pmace_data_fit(ctx, &cost));
  std::printf("iteration %4d  data-fit cost %.6e\n", 0, cost);
  const int report = iters >= 10 ? iters / 5 : 1;
  double gpu_s = 0.0;
  for (int k = 0; k < iters; k += report) {
    const int m = k + report <= iters ? report : iters - k;
    const auto t0 = std::chrono::steady_clock::now();
    CHECK_PM(pmace_iterate(ctx, m));
    CHECK_PM(pmace_sync(ctx));
    gpu_s += std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    CHECK_PM(pmace_data_fit(ctx, &cost));
    std::printf("iteration %4d  data-fit cost %.6e\n", k + m, cost);
  }
  CHECK_PM(pmace_reconstruct(ctx, xh_d));
  std::vector<cf> xh(x.size());
  CHECK_HIP(hipMemcpyAsync(xh.data(), xh_d, xh.size() * sizeof(cf), hipMemcpyDeviceToHost, st));
  CHECK_HIP(hipStreamSynchronize(st));

  // NRMSE (eq. (17)) over the central region the scan covers well.
  std::complex<double> c(0.0, 0.0);
  double nx = 0.0, nh = 0.0;
  const int lo = off + np / 2, hi = off + (scan - 1) * step + np / 2;
  for (int r = lo; r < hi; ++r)
    for (int q = lo; q < hi; ++q) {
      const std::complex<double> a(xh[(size_t)r * n + q]), b(x[(size_t)r * n + q]);
      c += std::conj(b) * a;
      nx += std::norm(b);
      nh += std::norm(a);
    }
  const double e = std::sqrt(std::fmax(nh + nx - 2.0 * std::abs(c), 0.0) / nx);
  std::printf("{\"n\": %d, \"np\": %d, \"positions\": %d, \"iterations\": %d, \"nrmse\": %.6f, "
              "\"data_fit\": %.6e, \"patch_updates_per_s\": %.4e}\n",
              n, np, J, iters, e, cost, (double)J * iters / gpu_s);

  pmace_destroy(ctx);
  CHECK_HIP(hipFree(ws));
  CHECK_HIP(hipFree(sim_ws));
  CHECK_HIP(hipFree(x_d));
  CHECK_HIP(hipFree(d_d));
  CHECK_HIP(hipFree(pos_d));
  CHECK_HIP(hipFree(z_d));
  CHECK_HIP(hipFree(xh_d));
  CHECK_HIP(hipStreamDestroy(st));
  return e < 0.5 ? 0 : 4;
}
