// Exercise every C-ABI entry point of liboct, valid and invalid calls alike,
// in a build whose HOST code carries AddressSanitizer and UndefinedBehavior-
// Sanitizer instrumentation (the device code is unchanged).  Any sanitizer
// report aborts the process; an unexpected status is reported and counted.
// Exit status 0 means every call returned what its declaration promises and
// no sanitizer fired.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "oct.h"

namespace {

int g_checks = 0, g_fail = 0;

void expect(bool ok, const char* what) {
  ++g_checks;
  if (!ok) {
    ++g_fail;
    std::fprintf(stderr, "UNEXPECTED: %s (last error: %s)\n", what, oct_last_error());
  }
}
void ok(oct_status s, const char* what) { expect(s == OCT_OK, what); }
void bad(oct_status s, const char* what) {
  expect(s != OCT_OK, what);
  expect(oct_last_error() != nullptr && std::strlen(oct_last_error()) > 0, "an error message is set");
}

oct_geometry base_geom(int lat_dims, int64_t nz, int64_t nx, int64_t ny, int64_t nk, int64_t batch) {
  oct_geometry g{};
  g.lateral_dims = lat_dims;
  g.kb_width = 6;
  g.n_depth = nz;
  g.n_x = nx;
  g.n_y = ny;
  g.n_k = nk;
  g.batch = batch;
  g.k_min = 2.0 * M_PI / 0.9;
  g.k_max = 2.0 * M_PI / 0.75;
  g.dx = g.dy = 2.0;
  g.dz = 0.0;
  g.z_focus = -1.0;
  g.beam_waist = 5.0;
  g.disp_a = 1e-3;
  g.disp_b = 0.0;
  g.oversamp = 2.0;
  g.kb_beta = 0.0;
  g.model = OCT_MODEL_DIRECT;
  return g;
}

template <typename T>
T* dev_fill(size_t n, std::mt19937& rng, float scale = 1.f) {
  std::normal_distribution<float> nd(0.f, scale);
  std::vector<T> h(n);
  float* f = reinterpret_cast<float*>(h.data());
  for (size_t i = 0; i < n * sizeof(T) / sizeof(float); ++i) f[i] = nd(rng);
  T* d = nullptr;
  if (hipMalloc(&d, n * sizeof(T)) != hipSuccess) return nullptr;
  hipMemcpy(d, h.data(), n * sizeof(T), hipMemcpyHostToDevice);
  return d;
}

bool all_finite(const void* dptr, size_t nfloats) {
  std::vector<float> h(nfloats);
  hipMemcpy(h.data(), dptr, nfloats * sizeof(float), hipMemcpyDeviceToHost);
  for (float v : h)
    if (!std::isfinite(v)) return false;
  return true;
}

// every entry point on one geometry (valid calls) plus argument errors
void run_geometry(const oct_geometry& g, const uint8_t* mask, std::mt19937& rng, const char* tag) {
  std::fprintf(stderr, "[sanitize] %s\n", tag);
  oct_plan_t p = nullptr;
  ok(oct_plan_create(&g, mask, &p), "plan_create");
  if (!p) return;
  const size_t n_img = (size_t)g.batch * g.n_y * g.n_x * g.n_depth;   // complex
  const size_t n_meas = (size_t)g.batch * g.n_y * g.n_x * g.n_k;      // real
  float2* x = dev_fill<float2>(n_img, rng);
  float2* x2 = dev_fill<float2>(n_img, rng);
  float2* z = dev_fill<float2>(n_img, rng);
  float* y = dev_fill<float>(n_meas, rng);
  double* dres = nullptr;
  hipMalloc(&dres, 2 * sizeof(double));

  ok(oct_forward(p, x, y, nullptr), "forward");
  ok(oct_adjoint(p, y, z, nullptr), "adjoint");
  ok(oct_adjoint_paper(p, y, z, nullptr), "adjoint_paper");
  ok(oct_grad(p, x, y, z, dres, nullptr), "grad");
  expect(all_finite(z, 2 * n_img), "grad finite");
  for (int pen : {OCT_PEN_L1, OCT_PEN_TV, OCT_PEN_HAAR, OCT_PEN_DTCWT}) {
    const oct_status s = oct_prox(p, pen, 0.1, 1e-3, 10, 1, 0.0, x, z, nullptr, nullptr);
    ok(s, "prox");
  }
  bad(oct_prox(p, 17, 0.1, 1e-3, 10, 2, 0.0, x, z, nullptr, nullptr), "prox: unknown penalty");
  bad(oct_prox(p, OCT_PEN_TV, 0.1, 1e-3, 0, 2, 0.0, x, z, nullptr, nullptr), "prox: tv_inner 0");
  bad(oct_prox(p, OCT_PEN_HAAR, 0.1, 1e-3, 10, 2, 0.5, x, z, nullptr, nullptr), "prox: Haar with a bound");
  double L = 0.0;
  ok(oct_lipschitz(p, 5, 1, 0, &L, nullptr), "lipschitz");
  expect(L > 0.0 && std::isfinite(L), "lipschitz positive");
  bad(oct_lipschitz(p, 0, 1, 0, &L, nullptr), "lipschitz: 0 iterations");

  std::vector<double> obj(6);
  for (int pen : {OCT_PEN_L1, OCT_PEN_TV, OCT_PEN_HAAR, OCT_PEN_DTCWT}) {
    oct_solve_params prm{};
    prm.penalty = pen;
    prm.iters = 6;
    prm.tv_inner = 5;
    prm.haar_levels = 1;
    prm.power_iters = 5;
    prm.lambda = 1e-2;
    prm.delta = 0.0;
    oct_solve_report rep{};
    rep.objective = obj.data();
    ok(oct_mbir_solve(p, y, &prm, z, &rep, nullptr), "solve");
    expect(std::isfinite(obj[5]) && rep.delta_used > 0.0, "solve report");
  }
  {
    // resume: 3 iterations, then 3 more from the saved state
    oct_solve_params prm{};
    prm.penalty = OCT_PEN_L1;
    prm.iters = 3;
    prm.lambda = 1e-2;
    prm.delta = 1.0 / (1.05 * L);
    prm.z_prev_out = x2;
    ok(oct_mbir_solve(p, y, &prm, z, nullptr, nullptr), "solve (first half)");
    prm.x0 = z;
    prm.z_prev0 = x2;
    prm.k0 = 3;
    prm.z_prev_out = nullptr;
    ok(oct_mbir_solve(p, y, &prm, x, nullptr, nullptr), "solve (resumed)");
    prm.k0 = -1;
    bad(oct_mbir_solve(p, y, &prm, x, nullptr, nullptr), "solve: negative k0");
  }
  if (g.batch <= OCT_MAX_LAMBDA_ITEMS) {
    std::vector<double> lam(g.batch);
    for (int64_t b = 0; b < g.batch; ++b) lam[b] = 1e-3 * (b + 1);
    oct_solve_params prm{};
    prm.penalty = OCT_PEN_HAAR;
    prm.iters = 2;
    prm.haar_levels = 1;
    prm.delta = 1.0 / (1.05 * L);
    prm.lambda_item = lam.data();
    ok(oct_mbir_solve(p, y, &prm, z, nullptr, nullptr), "solve with per-item weights");
    lam[0] = -1.0;
    bad(oct_mbir_solve(p, y, &prm, z, nullptr, nullptr), "solve: negative per-item weight");
  }
  {
    oct_solve_params prm{};
    prm.penalty = OCT_PEN_L1;
    prm.iters = 0;
    bad(oct_mbir_solve(p, y, &prm, z, nullptr, nullptr), "solve: 0 iterations");
    bad(oct_mbir_solve(p, y, nullptr, z, nullptr, nullptr), "solve: null parameters");
  }
  for (int st = 0; st < 6; ++st)
    for (int pen : {OCT_PEN_L1, OCT_PEN_TV, OCT_PEN_HAAR}) ok(oct_run_stage(p, st, pen, y, nullptr), "run_stage");
  bad(oct_run_stage(p, 9, OCT_PEN_L1, y, nullptr), "run_stage: unknown stage");
  for (int kind = 0; kind < 4; ++kind) ok(oct_direct(p, kind, y, z, nullptr), "direct");
  bad(oct_direct(p, 7, y, z, nullptr), "direct: unknown kind");
  double r = 0.0;
  ok(oct_ncc(p, x, z, &r, nullptr), "ncc");
  expect(std::fabs(r) <= 1.0 + 1e-12, "ncc in [-1, 1]");
  ok(oct_ncc_noalloc(x, z, (int64_t)n_img, dres, nullptr), "ncc_noalloc");
  bad(oct_ncc_noalloc(x, z, 0, dres, nullptr), "ncc_noalloc: n = 0");
  bad(oct_forward(p, nullptr, y, nullptr), "forward: null image");
  hipDeviceSynchronize();
  hipFree(x);
  hipFree(x2);
  hipFree(z);
  hipFree(y);
  hipFree(dres);
  ok(oct_plan_destroy(p), "plan_destroy");
}

}  // namespace

int main() {
  std::mt19937 rng(7);
  // host-only calls
  for (int which = 0; which < 4; ++which) {
    float h[64];
    int32_t n = 64;
    ok(oct_dtcwt_filter(which, h, &n), "dtcwt_filter");
    expect(n > 0 && n <= 64, "dtcwt_filter length");
  }
  {
    float h[64];
    int32_t n = 64;
    bad(oct_dtcwt_filter(4, h, &n), "dtcwt_filter: which = 4");
    bad(oct_dtcwt_filter(0, nullptr, &n), "dtcwt_filter: null output");
  }
  oct_geometry gb = base_geom(1, 256, 96, 1, 256, 2);
  expect(oct_plan_footprint_bytes(&gb, OCT_PEN_TV) > 0, "footprint");
  expect(oct_plan_footprint_bytes(&gb, -1) >= oct_plan_footprint_bytes(&gb, OCT_PEN_HAAR), "footprint bound");
  // invalid geometries are rejected before any device work
  {
    oct_plan_t p = nullptr;
    oct_geometry g = gb;
    g.n_depth = 0;
    bad(oct_plan_create(&g, nullptr, &p), "plan_create: n_depth 0");
    g = gb;
    g.kb_width = 5;
    bad(oct_plan_create(&g, nullptr, &p), "plan_create: J = 5");
    g = gb;
    g.k_max = g.k_min;
    bad(oct_plan_create(&g, nullptr, &p), "plan_create: empty band");
    g = gb;
    g.oversamp = 1.3;
    bad(oct_plan_create(&g, nullptr, &p), "plan_create: non-integer K");
    g = gb;
    g.lateral_dims = 3;
    bad(oct_plan_create(&g, nullptr, &p), "plan_create: 3 lateral axes");
    bad(oct_plan_create(nullptr, nullptr, &p), "plan_create: null geometry");
    bad(oct_plan_create(&gb, nullptr, nullptr), "plan_create: null output");
  }
  // B-scans (with a mask, ragged sizes, the literal model), a volume
  std::vector<uint8_t> mask((size_t)gb.n_x * gb.n_k);
  std::bernoulli_distribution half(0.5);
  for (auto& m : mask) m = half(rng) ? 1 : 0;
  run_geometry(gb, mask.data(), rng, "B-scan 256 x 96 x 256, batch 2, 50% mask");
  run_geometry(base_geom(1, 200, 56, 1, 196, 1), nullptr, rng, "B-scan 200 x 56 x 196");
  {
    oct_geometry g = base_geom(1, 128, 64, 1, 256, 1);
    g.model = OCT_MODEL_LITERAL;
    run_geometry(g, nullptr, rng, "B-scan 128 x 64 x 256, literal model");
  }
  run_geometry(base_geom(2, 128, 16, 16, 128, 1), nullptr, rng, "volume 128 x 16 x 16");
  {
    // nothing observed (all-zero mask): Phi = 0, the power iteration gives
    // exactly 0, a solve without a step size takes delta = 1 and returns 0
    const oct_geometry g = base_geom(1, 64, 16, 1, 64, 1);
    const std::vector<uint8_t> none((size_t)g.n_x * g.n_k, 0);
    oct_plan_t p = nullptr;
    ok(oct_plan_create(&g, none.data(), &p), "plan_create (nothing observed)");
    if (p) {
      const size_t n_img = (size_t)g.n_x * g.n_depth, n_meas = (size_t)g.n_x * g.n_k;
      float* y = dev_fill<float>(n_meas, rng);
      float2* z = dev_fill<float2>(n_img, rng);
      double L = -1.0;
      ok(oct_lipschitz(p, 5, 1, 0, &L, nullptr), "lipschitz (nothing observed)");
      expect(L == 0.0, "lipschitz is exactly 0 when nothing is observed");
      for (int pen : {OCT_PEN_L1, OCT_PEN_TV, OCT_PEN_HAAR}) {
        oct_solve_params prm{};
        prm.penalty = pen;
        prm.iters = 4;
        prm.tv_inner = 5;
        prm.haar_levels = 2;
        prm.power_iters = 5;
        prm.lambda = 1e-2;
        prm.delta = 0.0;
        oct_solve_report rep{};
        ok(oct_mbir_solve(p, y, &prm, z, &rep, nullptr), "solve (nothing observed)");
        expect(rep.lipschitz_est == 0.0 && rep.delta_used == 1.0, "nothing observed: L = 0, delta = 1");
        std::vector<float> h(2 * n_img);
        hipMemcpy(h.data(), z, h.size() * sizeof(float), hipMemcpyDeviceToHost);
        bool zero = true;
        for (float v : h) zero = zero && v == 0.f;
        expect(zero, "nothing observed: the solution is exactly zero");
      }
      hipFree(y);
      hipFree(z);
      ok(oct_plan_destroy(p), "plan_destroy (nothing observed)");
    }
  }
  {
    // released plan memory is reused by the next plan
    oct_plan_t p = nullptr;
    ok(oct_plan_create(&gb, nullptr, &p), "plan_create (release)");
    if (p) ok(oct_plan_release(p), "plan_release");
    hipDeviceSynchronize();
  }
  std::fprintf(stderr, "[sanitize] %d checks, %d unexpected\n", g_checks, g_fail);
  std::printf("%s %d %d\n", g_fail == 0 ? "PASS" : "FAIL", g_checks, g_fail);
  return g_fail == 0 ? 0 : 1;
}
