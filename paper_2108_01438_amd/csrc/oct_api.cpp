// Host side of liboct: plan construction (FP64 tables), argument validation
// and the orchestration of the kernels behind the C ABI in include/oct.h.
#include "../../include/oct.h"
#include "oct_common.h"
#include "oct_fft.h"

#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

namespace {

thread_local std::string g_err;

oct_status fail(oct_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

#define HIPCHK(expr)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess) return fail(OCT_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

constexpr double kPi = 3.14159265358979323846;

// Modified Bessel function I0 by its power series sum_k ((x/2)^k / k!)^2.
double bessel_i0(double x) {
  const double q = 0.25 * x * x;
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 500; ++k) {
    term *= q / ((double)k * k);
    sum += term;
    if (term < 1e-17 * sum) break;
  }
  return sum;
}

// Zero-edge Kaiser-Bessel window and its continuous Fourier transform.
double kb0(double u, int J, double b) {
  const double s = 1.0 - (2.0 * u / J) * (2.0 * u / J);
  if (s < 0.0) return 0.0;
  return (bessel_i0(b * std::sqrt(s)) - 1.0) / (bessel_i0(b) - 1.0);
}

double kb0_ft(double f, int J, double b) {
  const double w = kPi * J * f;
  const double a2 = b * b - w * w;
  double sh;
  if (a2 > 0) {
    const double a = std::sqrt(a2);
    sh = J * std::sinh(a) / a;
  } else if (a2 < 0) {
    const double a = std::sqrt(-a2);
    sh = J * std::sin(a) / a;
  } else {
    sh = J;
  }
  const double box = (w == 0.0) ? (double)J : J * std::sin(w) / w;
  return (sh - box) / (bessel_i0(b) - 1.0);
}

// Tap j of the J-tap window as a polynomial in x = 2 f - 1, f = frac(t):
// Chebyshev interpolation at KB_DEG+1 nodes, converted to monomials.  Only
// taps j < J/2 are stored, split into even and odd parts in x^2: the window
// is even, so tap J-1-j is the same polynomial at -x.
void kb_pieces(int J, double b, std::vector<float>& out) {
  const int D = OCT_KB_DEG;
  const int Hh = (D + 1) / 2;
  out.assign((size_t)(J / 2) * 2 * Hh, 0.f);
  for (int j = 0; j < J / 2; ++j) {
    std::vector<double> c(D + 1, 0.0);
    for (int k = 0; k <= D; ++k) {
      double s = 0.0;
      for (int i = 0; i <= D; ++i) {
        const double th = kPi * (i + 0.5) / (D + 1);
        const double x = std::cos(th);
        const double f = 0.5 * (x + 1.0);
        s += kb0(f + J / 2 - 1 - j, J, b) * std::cos(k * th);
      }
      c[k] = s * (k == 0 ? 1.0 : 2.0) / (D + 1);
    }
    // Chebyshev -> monomial: accumulate T_k coefficients
    std::vector<double> mono(D + 1, 0.0), tkm1(D + 1, 0.0), tk(D + 1, 0.0), tkp1(D + 1, 0.0);
    tkm1[0] = 1.0;          // T0
    tk[1] = 1.0;            // T1
    for (int i = 0; i <= D; ++i) mono[i] += c[0] * tkm1[i];
    for (int i = 0; i <= D; ++i) mono[i] += c[1] * tk[i];
    for (int k = 2; k <= D; ++k) {
      std::fill(tkp1.begin(), tkp1.end(), 0.0);
      for (int i = 0; i < D; ++i) tkp1[i + 1] += 2.0 * tk[i];
      for (int i = 0; i <= D; ++i) tkp1[i] -= tkm1[i];
      for (int i = 0; i <= D; ++i) mono[i] += c[k] * tkp1[i];
      tkm1 = tk;
      tk = tkp1;
    }
    for (int i = 0; i < Hh; ++i) {
      out[(size_t)j * 2 * Hh + i] = (float)mono[2 * i];
      out[(size_t)j * 2 * Hh + Hh + i] = (float)mono[2 * i + 1];
    }
  }
}

bool factorize(int n, FftDesc& d) {
  std::memset(&d, 0, sizeof(d));
  d.n = n;
  if (n < 1) return false;
  // powers of two as radix 8 with a 4 (or 4 x 4) instead of a trailing 2
  int m = n, a = 0;
  while (m % 2 == 0) { m /= 2; ++a; }
  std::vector<int> rad;
  const int q = a / 3, r = a % 3;
  if (r == 1 && q >= 1) {
    for (int i = 0; i < q - 1; ++i) rad.push_back(8);
    rad.push_back(4);
    rad.push_back(4);
  } else {
    for (int i = 0; i < q; ++i) rad.push_back(8);
    if (r == 1) rad.push_back(2);
    if (r == 2) rad.push_back(4);
  }
  for (int p : {5, 3, 7})
    while (m % p == 0) { m /= p; rad.push_back(p); }
  if (m != 1 || (int)rad.size() > OCT_MAX_STAGES) return false;
  int prod = 1, mr = 8;
  for (size_t s = 0; s < rad.size(); ++s) {
    d.radix[s] = rad[s];
    d.ns[s] = prod;
    d.div_nb[s] = make_fastdiv((uint32_t)(n / rad[s]));
    d.div_ns[s] = make_fastdiv((uint32_t)prod);
    prod *= rad[s];
    if (rad[s] < mr) mr = rad[s];
  }
  d.nstages = (int)rad.size();
  d.min_radix = mr;
  return true;
}

// Per-stage twiddle rows of FftDesc (layout in oct_common.h), built in FP64.
std::vector<float2> twiddles(FftDesc& d) {
  std::vector<float2> t;
  for (int s = 0; s < d.nstages; ++s) {
    const int R = d.radix[s], Ns = d.ns[s], P = fft_tw_pad(R);
    d.tw_off[s] = (int)t.size();
    if (Ns == 1) continue;   // first stage: all factors are 1
    for (int k = 0; k < Ns; ++k)
      for (int r = 1; r <= P; ++r) {
        float2 w = make_float2(0.f, 0.f);
        if (r < R) {
          const double a = -2.0 * kPi * (double)(r * k) / (double)(Ns * R);
          w = make_float2((float)std::cos(a), (float)std::sin(a));
        }
        t.push_back(w);
      }
  }
  d.tw_total = (int)t.size();
  if (t.empty()) t.push_back(make_float2(0.f, 0.f));   // keep the device table non-empty
  return t;
}

}  // namespace

struct oct_plan {
  oct_geometry g{};
  int device = 0;
  int lat_dims = 1;
  int64_t Nz = 0, Nx = 0, Ny = 1, Mk = 0, B = 1, Nlat = 0, K = 0;
  int nc = 0, J = 6;
  double dk = 0, dz = 0, zf = 0, kbb = 0, ct = 0, df = 0;
  FftDesc fK{}, fX{}, fY{}, fM{};
  float2 *twK = nullptr, *twX = nullptr, *twY = nullptr;
  float2* twM = nullptr;         // spectral-axis transform (analytic signal; literal chain's D)
  float2* tv_last = nullptr;     // the TV dual the last solve ended with (p0 or p1), for a resumed solve
  // literal K, Q, D chain (model 1): even-pixel NUFFT tables, the N-point transform, e^{j Omega}
  int model = OCT_MODEL_DIRECT;
  // half-spectrum path (direct model): the forward NUFFT keeps W_h(q) =
  // (W(q) + conj W(-q)) / 2 for q_x <= n_x / 2 only; column pairs (q, -q)
  bool hs = false;
  int64_t Nxh = 0;               // n_x / 2 + 1
  int64_t Nxs = 0;               // half-spectrum slot stride per y row (n_x; slots < Nxh used)
  int64_t X1s = 0;               // column stride of X1's y rows (n_x, or n_x + 1 for a volume)
  int4* pairs = nullptr;
  int n_pairs = 0;
  // every measurement pixel observed (no mask, or a mask of all ones): on the
  // half-spectrum path the residual seam reduces to R^ = W_h / N_lat - Y_h
  bool full = true;
  float2* yhat = nullptr;        // Y_h = F_lat(y) / N_lat of the running solve (W's layout), first use
  FftDesc fN{};
  float2* twN = nullptr;
  double* k2x4e = nullptr;       // [N] 4 k_{2j}^2
  float2* phase_e = nullptr;     // [N] e^{-j 2 k_{2j} z_f}
  float2* omph = nullptr;        // [Mk] e^{j Omega_m}
  float2* Wn = nullptr;          // [batch][lat][N] samples of K
  float* deap = nullptr;
  double* k2x4 = nullptr;
  float2* phase = nullptr;
  double* q2 = nullptr;
  float* beam = nullptr;
  float* kbc = nullptr;
  uint32_t* mask = nullptr;
  int mask_words = 0;

  float2 *X1 = nullptr, *W = nullptr;
  double* partial = nullptr;
  int partial_cap = 0;
  double* dscal = nullptr;       // device scalars
  // direct reconstructions: lateral-frequency-zero tables and the filled spectrum
  double* q2zero = nullptr;      // [Nlat] zeros
  float* beamone = nullptr;      // [Nlat] ones
  float2* phase_nd = nullptr;    // [Mk] e^{-j 2 k_m z_f} (no dispersion phase)
  float* yfill = nullptr;        // [batch][lat][Mk] real spectra (filled / residual), allocated on first use
  float* yitem = nullptr;        // [batch][lat][Mk] measurements scaled per item (per-item weights), first use
  // solver state, allocated on first use
  float2 *za = nullptr, *zb = nullptr;
  float2* xext = nullptr;        // the extrapolated point x of the current iteration (lat_fwd -> update)
  float2 *p0 = nullptr, *p1 = nullptr, *tvwork = nullptr;
  float2* dtwork = nullptr;      // DT-CWT trees and staging (8 images; 24 for a volume)
  double* hist = nullptr;
  int hist_cap = 0;
  std::vector<void*> allocs;

  int64_t n_img() const { return B * Nlat * Nz; }
  int64_t n_meas() const { return B * Nlat * Mk; }
};

namespace {

// Plan memory comes from the device's stream-ordered pool on the null stream
// (allocated ready for use: the null stream is synchronised), so that a plan
// can be freed without synchronising the device (oct_plan_release).  The
// pool keeps freed blocks for the next plans (release threshold raised once
// per device).
void keep_pool_memory(int device) {
  static std::mutex mu;
  static bool done[64] = {};
  std::lock_guard<std::mutex> lock(mu);
  if (device < 0 || device >= 64 || done[device]) return;
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, device) == hipSuccess) {
    uint64_t thr = UINT64_MAX;
    hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
  done[device] = true;
}

template <typename T>
oct_status dev_alloc(oct_plan* p, T** out, size_t count) {
  void* ptr = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMallocAsync(&ptr, count * sizeof(T), nullptr);
  if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  if (e != hipSuccess) return fail(OCT_E_NOMEM, std::string("hipMallocAsync: ") + hipGetErrorString(e));
  p->allocs.push_back(ptr);
  *out = reinterpret_cast<T*>(ptr);
  return OCT_OK;
}

template <typename T>
oct_status upload(oct_plan* p, T** out, const std::vector<T>& h) {
  oct_status s = dev_alloc(p, out, h.size());
  if (s != OCT_OK) return s;
  HIPCHK(hipMemcpy(*out, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  return OCT_OK;
}

#define OCTCHK(expr)                \
  do {                              \
    oct_status s_ = (expr);         \
    if (s_ != OCT_OK) return s_;    \
  } while (0)

oct_status validate(const oct_geometry* g) {
  if (!g) return fail(OCT_E_INVALID, "geometry is NULL");
  if (g->lateral_dims != 1 && g->lateral_dims != 2) return fail(OCT_E_INVALID, "lateral_dims must be 1 or 2");
  if (g->n_depth < 2 || g->n_x < 1 || g->n_y < 1 || g->n_k < 2 || g->batch < 1)
    return fail(OCT_E_INVALID, "sizes must be positive (n_depth, n_k >= 2)");
  if (g->lateral_dims == 1 && g->n_y != 1) return fail(OCT_E_INVALID, "a B-scan has n_y = 1");
  if (!(g->k_max > g->k_min) || !(g->k_min > 0)) return fail(OCT_E_INVALID, "need 0 < k_min < k_max");
  if (!(g->dx > 0) || (g->lateral_dims == 2 && !(g->dy > 0))) return fail(OCT_E_INVALID, "lateral pitch must be > 0");
  if (g->kb_width != 4 && g->kb_width != 6 && g->kb_width != 8)
    return fail(OCT_E_INVALID, "kb_width must be 4, 6 or 8");
  if (g->model != OCT_MODEL_DIRECT && g->model != OCT_MODEL_LITERAL) return fail(OCT_E_INVALID, "unknown model");
  if (g->model == OCT_MODEL_LITERAL && g->n_k != 2 * g->n_depth)
    return fail(OCT_E_INVALID, "the literal chain needs n_k = 2 n_depth");
  if (!(g->oversamp >= 1.0)) return fail(OCT_E_INVALID, "oversamp must be >= 1");
  const double Kf = g->oversamp * (double)g->n_depth;
  if (std::fabs(Kf - std::round(Kf)) > 1e-9) return fail(OCT_E_INVALID, "oversamp * n_depth must be an integer");
  if (std::llround(Kf) < 2 * g->kb_width) return fail(OCT_E_INVALID, "oversampled grid must hold at least 2 J cells");
  return OCT_OK;
}

oct_status unsupported_sizes(const oct_geometry* g) {
  const int64_t K = (int64_t)std::llround(g->oversamp * (double)g->n_depth);
  FftDesc d;
  if (K > 8192) return fail(OCT_E_UNSUPPORTED, "oversampled grid K > 8192");
  if (!factorize((int)K, d)) return fail(OCT_E_UNSUPPORTED, "K has a prime factor above 7");
  if (g->n_x > 4096 || !factorize((int)g->n_x, d)) return fail(OCT_E_UNSUPPORTED, "n_x must be 7-smooth and <= 4096");
  if (g->lateral_dims == 2 && (g->n_y > 4096 || !factorize((int)g->n_y, d)))
    return fail(OCT_E_UNSUPPORTED, "n_y must be 7-smooth and <= 4096");
  if (g->n_k > 8192) return fail(OCT_E_UNSUPPORTED, "n_k > 8192");
  if (g->model == OCT_MODEL_LITERAL) {
    FftDesc fn, fm;
    if (!factorize((int)g->n_depth, fn) || !factorize((int)g->n_k, fm))
      return fail(OCT_E_UNSUPPORTED, "the literal chain needs a 7-smooth n_depth");
    bool one;
    if (literal_dq_threads(fn, fm, &one) == 0)
      return fail(OCT_E_UNSUPPORTED, "n_k has too many radix-2/3 butterflies per stage");
  }
  // the kernels' compile-time FFT paths must use the radix plan of factorize
  {
    constexpr int sizes[] = {OCT_CT_K_SIZES, OCT_CT_LAT_SIZES};
    for (int n : sizes) {
      FftDesc f;
      factorize(n, f);
      const CtPlan c = ct_plan(n);
      bool same = c.ns == f.nstages;
      for (int s = 0; same && s < c.ns; ++s) same = c.r[s] == f.radix[s];
      if (!same) return fail(OCT_E_UNSUPPORTED, "internal: compile-time FFT plan differs from the host plan");
    }
  }
  // every FFT stage must fit the butterflies-per-thread limit of a 1024-thread block
  for (int64_t n : {K, g->n_x, g->lateral_dims == 2 ? g->n_y : (int64_t)1}) {
    FftDesc f;
    factorize((int)n, f);
    if (f.nstages > 0 && n / f.min_radix > (int64_t)fft_maxb(f) * 1024)
      return fail(OCT_E_UNSUPPORTED, "transform length has too many radix-2/3 butterflies per stage");
  }
  // adjoint column kernel keeps the grid or the samples in LDS
  const size_t lds = (size_t)K * 8 + (size_t)g->n_k * 14 + 4096;
  if (lds > 160 * 1024 - 4096) return fail(OCT_E_UNSUPPORTED, "grid + samples exceed the LDS of one CU");
  // base cells of one column are stored as 16-bit offsets: bound the span of t
  const double dk = (g->k_max - g->k_min) / (double)(g->n_k - 1);
  const double dz = g->dz > 0 ? g->dz : kPi / (2.0 * (double)g->n_depth * dk);
  const double tmax = (double)K * dz / (2.0 * kPi) * 2.0 * g->k_max;
  if (tmax + 2 * g->kb_width > 32000.0)
    return fail(OCT_E_UNSUPPORTED, "oversampled-grid coordinates span more than 32000 cells");
  return OCT_OK;
}

LineGeom lines_x(const oct_plan* p, int rows) {
  LineGeom lg{};
  lg.L = (int)p->Nx;
  lg.rows = rows;
  lg.n_lines = (int)(p->B * p->Ny);
  lg.ocnt = 1;
  lg.sa = p->Nx * rows;
  lg.sb = 0;
  lg.es = rows;
  lg.lat_lines = (int)p->Ny;
  return lg;
}

LineGeom lines_y(const oct_plan* p, int rows) {
  LineGeom lg{};
  lg.L = (int)p->Ny;
  lg.rows = rows;
  lg.n_lines = (int)(p->B * p->Nx);
  lg.ocnt = (int)p->Nx;
  lg.sa = p->Ny * p->Nx * rows;
  lg.sb = rows;
  lg.es = p->Nx * rows;
  lg.lat_lines = 1;
  return lg;
}

// y lines of a half-spectrum array [batch][n_y][n_x/2 + 1][rows]
// y lines of X1 (y rows X1s columns apart)
LineGeom lines_y_x1(const oct_plan* p, int rows) {
  LineGeom lg = lines_y(p, rows);
  lg.sa = p->Ny * p->X1s * rows;
  lg.es = p->X1s * rows;
  return lg;
}

LineGeom lines_y_half(const oct_plan* p, int rows) {
  LineGeom lg = lines_y(p, rows);
  lg.n_lines = (int)(p->B * p->Nxh);
  lg.ocnt = (int)p->Nxh;
  lg.sa = p->Ny * p->Nxs * rows;
  lg.es = p->Nxs * rows;
  return lg;
}

LatArgs lat_args(const oct_plan* p, const LineGeom& lg, bool yaxis) {
  LatArgs a{};
  a.lg = lg;
  a.fd = yaxis ? p->fY : p->fX;
  a.tw = yaxis ? p->twY : p->twX;
  int nthr = 256, rs = lg.L;
  a.T = lateral_pick_tile(lg, a.fd, &nthr, &rs);
  a.log2T = 0;
  while ((1 << a.log2T) < a.T) ++a.log2T;
  a.rowstride = rs;
  a.n_tiles = (lg.rows + a.T - 1) / a.T;
  a.scale = 1.f;
  a.scale2 = 1.f;
  a.bound = INFINITY;
  a.mask = p->mask;
  a.mask_words = p->mask_words;
  return a;
}

int lat_blocks(const LatArgs& a) { return a.lg.n_lines * a.n_tiles; }

NufftArgs nufft_args(const oct_plan* p) {
  NufftArgs a{};
  a.Nz = (int)p->Nz;
  a.Mk = (int)p->Mk;
  a.K = (int)p->K;
  a.nc = p->nc;
  a.J = p->J;
  a.Nlat = (int)p->Nlat;
  a.n_cols = (int)(p->B * p->Nlat);
  a.Nx = (int)p->Nx;
  a.xs = (int)p->X1s;
  a.ct = p->ct;
  a.invK = 1.0 / (double)p->K;
  a.df = p->df;
  a.k_min = p->g.k_min;
  a.dk = p->dk;
  a.k2x4 = p->k2x4;
  a.phase = p->phase;
  a.q2 = p->q2;
  a.beam = p->beam;
  a.deap = p->deap;
  a.kbc = p->kbc;
  a.fK = p->fK;
  a.twK = p->twK;
  a.pairs = p->pairs;
  a.n_pairs = p->n_pairs;
  a.n_half = (int)(p->Ny * p->Nxs);
  return a;
}

hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

// NUFFT column arguments of the literal chain's K: the N even detector
// wavenumbers k_{2j} = k_min + 2 j dk, the focus phase without Omega
NufftArgs even_args(const oct_plan* p) {
  NufftArgs a = nufft_args(p);
  a.Mk = (int)p->Nz;
  a.dk = 2.0 * p->dk;
  a.k2x4 = p->k2x4e;
  a.phase = p->phase_e;
  return a;
}

// X1 (lateral spectra of the image) -> W (spectra at the detector pixels)
oct_status run_cols_fwd(oct_plan* p, hipStream_t s, bool half) {
  if (half) {
    HIPCHK(launch_nufft_fwd_pair(nufft_args(p), p->X1, p->W, s));
    return OCT_OK;
  }
  if (p->model == OCT_MODEL_DIRECT) {
    HIPCHK(launch_nufft_fwd(nufft_args(p), p->X1, p->W, s));
    return OCT_OK;
  }
  HIPCHK(launch_nufft_fwd(even_args(p), p->X1, p->Wn, s));
  HIPCHK(launch_literal_dq(false, p->Wn, p->W, p->omph, (int)p->Nz, p->B * p->Nlat, p->fN, p->twN, p->fM, p->twM,
                           s));
  return OCT_OK;
}

// W -> X1 (the exact adjoint of run_cols_fwd)
oct_status run_cols_adj(oct_plan* p, hipStream_t s, bool half) {
  if (half) {
    HIPCHK(launch_nufft_adj_pair(nufft_args(p), p->W, p->X1, s));
    return OCT_OK;
  }
  if (p->model == OCT_MODEL_DIRECT) {
    HIPCHK(launch_nufft_adj(nufft_args(p), p->W, p->X1, s));
    return OCT_OK;
  }
  HIPCHK(launch_literal_dq(true, p->W, p->Wn, p->omph, (int)p->Nz, p->B * p->Nlat, p->fN, p->twN, p->fM, p->twM,
                           s));
  HIPCHK(launch_nufft_adj(even_args(p), p->Wn, p->X1, s));
  return OCT_OK;
}

// x (image, or z + mu (z - zo) when z != NULL, then also stored to xout when
// that is not NULL) -> X1 = F_lat x
oct_status run_lat_forward(oct_plan* p, const float2* x, const float2* z, const float2* zo, float mu, hipStream_t s,
                           float2* xout = nullptr) {
  LatArgs a = lat_args(p, lines_x(p, (int)p->Nz), false);
  a.src = x;
  a.z = z;
  a.zo = const_cast<float2*>(zo);
  a.mu = mu;
  a.xout = xout;
  a.dst = p->X1;
  a.sa_out = p->X1s * p->Nz;   // X1's x lines (image rows: lg.sa)
  HIPCHK(launch_lateral(LAT_FFT, a, s));
  if (p->lat_dims == 2) {
    LatArgs b = lat_args(p, lines_y_x1(p, (int)p->Nz), true);
    b.src = p->X1;
    b.dst = p->X1;
    HIPCHK(launch_lateral(LAT_FFT, b, s));
  }
  return OCT_OK;
}

// W (after the NUFFT) -> y = s . Re(F_lat^{-1} W)
oct_status run_meas_forward(oct_plan* p, float* y, hipStream_t s, bool half) {
  const int rows = (int)p->Mk;
  if (p->lat_dims == 2) {
    LatArgs b = lat_args(p, half ? lines_y_half(p, rows) : lines_y(p, rows), true);
    b.src = p->W;
    b.dst = p->W;
    b.inverse = 1;
    b.scale = 1.f / (float)p->Ny;
    HIPCHK(launch_lateral(LAT_FFT, b, s));
  }
  LatArgs a = lat_args(p, lines_x(p, rows), false);
  if (half) a.sa_half = p->Nxs * rows;
  a.src = p->W;
  a.dstf = y;
  a.inverse = 1;
  a.scale = 1.f / (float)p->Nx;
  HIPCHK(launch_lateral(LAT_FWD_MEAS, a, s));
  return OCT_OK;
}

// r -> W = F_lat(s . r) / N_lat (into dst, W's layout, when given)
oct_status run_meas_adjoint(oct_plan* p, const float* r, hipStream_t s, bool half, bool use_mask = true,
                            float2* dst = nullptr) {
  const int rows = (int)p->Mk;
  if (!dst) dst = p->W;
  LatArgs a = lat_args(p, lines_x(p, rows), false);
  if (half) a.sa_half = p->Nxs * rows;
  if (!use_mask) a.mask = nullptr;
  a.srcf = r;
  a.dst = dst;
  a.scale = 1.f / (float)p->Nx;
  HIPCHK(launch_lateral(LAT_ADJ_MEAS, a, s));
  if (p->lat_dims == 2) {
    LatArgs b = lat_args(p, half ? lines_y_half(p, rows) : lines_y(p, rows), true);
    b.src = dst;
    b.dst = dst;
    b.scale = 1.f / (float)p->Ny;
    HIPCHK(launch_lateral(LAT_FFT, b, s));
  }
  return OCT_OK;
}

// r -> W = F_lat A(s . r) / N_lat, A(z) = conj of the analytic signal along k (eq. (10)-(11))
oct_status ensure_analytic(oct_plan* p) {
  if (p->twM) return OCT_OK;
  FftDesc f;
  if (p->Mk > 8192 || !factorize((int)p->Mk, f))
    return fail(OCT_E_UNSUPPORTED, "the analytic signal needs a 7-smooth n_k <= 8192");
  if (p->Mk / f.min_radix > (int64_t)fft_maxb(f) * 1024)
    return fail(OCT_E_UNSUPPORTED, "n_k has too many radix-2/3 butterflies per stage");
  OCTCHK(upload(p, &p->twM, twiddles(f)));
  p->fM = f;
  return OCT_OK;
}

oct_status run_meas_backward_paper(oct_plan* p, const float* r, hipStream_t s) {
  OCTCHK(ensure_analytic(p));
  HIPCHK(launch_analytic_conj(r, p->mask, p->mask_words, (int)p->Mk, (int)p->Nlat, p->B * p->Nlat, p->fM, p->twM,
                              p->W, s));
  LatArgs a = lat_args(p, lines_x(p, (int)p->Mk), false);
  a.src = p->W;
  a.dst = p->W;
  a.scale = 1.f / (float)p->Nx;
  HIPCHK(launch_lateral(LAT_FFT, a, s));
  if (p->lat_dims == 2) {
    LatArgs b = lat_args(p, lines_y(p, (int)p->Mk), true);
    b.src = p->W;
    b.dst = p->W;
    b.scale = 1.f / (float)p->Ny;
    HIPCHK(launch_lateral(LAT_FFT, b, s));
  }
  return OCT_OK;
}

// W -> W = F_lat A(s . (Re F_lat^{-1} W - y)) / N_lat with per-block sum r^2 (the paper's
// backward operator in the normal seam); the real residual goes through yfill
oct_status run_normal_paper(oct_plan* p, const float* y, double* partial, int* nparts, hipStream_t s) {
  if (!p->yfill) OCTCHK(dev_alloc(p, &p->yfill, (size_t)p->n_meas()));
  if (p->lat_dims == 2) {
    LatArgs b = lat_args(p, lines_y(p, (int)p->Mk), true);
    b.src = p->W;
    b.dst = p->W;
    b.inverse = 1;
    b.scale = 1.f / (float)p->Ny;
    HIPCHK(launch_lateral(LAT_FFT, b, s));
  }
  LatArgs a = lat_args(p, lines_x(p, (int)p->Mk), false);
  a.src = p->W;
  a.dstf = p->yfill;
  a.y = y;
  a.inverse = 1;
  a.scale = 1.f / (float)p->Nx;
  a.partial = partial;
  if (nparts) *nparts = lat_blocks(a);
  HIPCHK(launch_lateral(LAT_RESID, a, s));
  return run_meas_backward_paper(p, p->yfill, s);
}

// W -> W = F_lat(s . (Re F_lat^{-1} W - y)) / N_lat with per-block sum r^2; returns #partials
oct_status run_normal(oct_plan* p, const float* y, double* partial, int* nparts, hipStream_t s, bool half) {
  const int rows = (int)p->Mk;
  if (p->lat_dims == 2) {
    LatArgs b = lat_args(p, half ? lines_y_half(p, rows) : lines_y(p, rows), true);
    b.src = p->W;
    b.dst = p->W;
    b.inverse = 1;
    b.scale = 1.f / (float)p->Ny;
    HIPCHK(launch_lateral(LAT_FFT, b, s));
  }
  LatArgs a = lat_args(p, lines_x(p, rows), false);
  if (half) a.sa_half = p->Nxs * rows;
  a.src = p->W;
  a.dst = p->W;
  a.y = y;
  a.inverse = 1;
  a.scale = 1.f / (float)p->Nx;
  a.scale2 = 1.f / (float)p->Nx;
  a.partial = partial;
  if (nparts) *nparts = lat_blocks(a);
  HIPCHK(launch_lateral(LAT_NORMAL, a, s));
  if (p->lat_dims == 2) {
    LatArgs b = lat_args(p, half ? lines_y_half(p, rows) : lines_y(p, rows), true);
    b.src = p->W;
    b.dst = p->W;
    b.scale = 1.f / (float)p->Ny;
    HIPCHK(launch_lateral(LAT_FFT, b, s));
  }
  return OCT_OK;
}

// The normal seam of a fully observed half-spectrum plan: X1 -> W = R^ =
// W_h / N_lat - yh in the forward pair kernel (yh: Y_h = F_lat(y) / N_lat in
// W's layout, possibly W itself; NULL for y = 0), the per-block sums of r^2
// into partial when that is not NULL; returns #partials.
bool spectral_seam(const oct_plan* p, bool paper) { return p->hs && p->full && !paper; }

oct_status run_cols_fwd_res(oct_plan* p, const float2* yh, double* partial, int* nparts, hipStream_t s) {
  HIPCHK(launch_nufft_fwd_pair_res(nufft_args(p), p->X1, p->W, yh, partial, s));
  if (nparts) *nparts = (int)(p->n_pairs * p->B);
  return OCT_OK;
}

// X1 -> X1 = the adjoint columns of R^ = W_h / N_lat - yh: the two column
// kernels with the spectral seam between them, in one launch when the pair
// fits it (R^ stays in registers), else the residual-writing forward kernel
// and the adjoint kernel over W
oct_status run_cols_normal(oct_plan* p, const float2* yh, double* partial, int* nparts, hipStream_t s) {
  const NufftArgs a = nufft_args(p);
  if (nufft_normal_pair_supported(a)) {
    HIPCHK(launch_nufft_normal_pair(a, p->X1, yh, partial, p->X1, s));
    if (nparts) *nparts = (int)(p->n_pairs * p->B);
    return OCT_OK;
  }
  OCTCHK(run_cols_fwd_res(p, yh, partial, nparts, s));
  HIPCHK(launch_nufft_adj_pair(a, p->W, p->X1, s));
  return OCT_OK;
}

// X1 (adjoint NUFFT output) -> g = F_lat^H X1 written to out
oct_status run_lat_adjoint(oct_plan* p, float2* out, hipStream_t s) {
  if (p->lat_dims == 2) {
    LatArgs b = lat_args(p, lines_y_x1(p, (int)p->Nz), true);
    b.src = p->X1;
    b.dst = p->X1;
    b.inverse = 1;
    HIPCHK(launch_lateral(LAT_FFT, b, s));
  }
  LatArgs a = lat_args(p, lines_x(p, (int)p->Nz), false);
  a.src = p->X1;
  a.sa_in = p->X1s * p->Nz;   // X1's x lines
  a.dst = out;
  a.inverse = 1;
  HIPCHK(launch_lateral(LAT_FFT, a, s));
  return OCT_OK;
}

int partial_need(oct_plan* p) {
  int need = 2048;
  const LatArgs a = lat_args(p, lines_x(p, (int)p->Mk), false);
  need = std::max(need, lat_blocks(a));
  const LatArgs b = lat_args(p, lines_x(p, (int)p->Nz), false);
  need = std::max(need, lat_blocks(b));
  ProxGeom pg{(int)p->B, (int)p->Ny, (int)p->Nx, (int)p->Nz, p->lat_dims};
  for (int lv = 1; lv <= 5; ++lv) need = std::max(need, haar_partials(pg, lv));
  need = std::max(need, tv_partials(pg, TV_MAX_TILED_INNER));
  need = std::max(need, tv_partials(pg, TV_MAX_TILED_INNER + 1));
  for (int lv = 1; lv <= (p->lat_dims == 1 ? 5 : 4); ++lv) need = std::max(need, dtcwt_partials(pg, lv));
  need = std::max(need, (int)(p->n_pairs * p->B));   // the residual partials of the spectral seam
  return need;
}

// Column stride of the y rows of the spectral buffers (see plan creation):
// a volume pads them by one column; the elements of W (the full spectrum, or
// the padded half spectrum if larger) and of X1.
static int64_t w_slot_stride(const oct_geometry& g) { return g.n_y > 1 ? g.n_x + 1 : g.n_x; }
static int64_t w_elems(const oct_geometry& g) {
  return g.batch * std::max(g.n_y * g.n_x, g.n_y * w_slot_stride(g)) * g.n_k;
}
static int64_t x1_elems(const oct_geometry& g) { return g.batch * g.n_y * w_slot_stride(g) * g.n_depth; }

oct_status ensure_solver_state(oct_plan* p, int pen, int iters) {
  const size_t n0 = p->allocs.size();
  if (!p->za) {
    OCTCHK(dev_alloc(p, &p->za, p->n_img()));
    OCTCHK(dev_alloc(p, &p->zb, p->n_img()));
    HIPCHK(hipMemset(p->za, 0, sizeof(float2) * p->n_img()));
    HIPCHK(hipMemset(p->zb, 0, sizeof(float2) * p->n_img()));
  }
  if (!p->xext) {
    OCTCHK(dev_alloc(p, &p->xext, p->n_img()));
    HIPCHK(hipMemset(p->xext, 0, sizeof(float2) * p->n_img()));
  }
  if (pen == OCT_PEN_TV && !p->p0) {
    const int nd = p->lat_dims + 1;
    OCTCHK(dev_alloc(p, &p->p0, (size_t)p->n_img() * nd));
    OCTCHK(dev_alloc(p, &p->p1, (size_t)p->n_img() * nd));
    ProxGeom pg{(int)p->B, (int)p->Ny, (int)p->Nx, (int)p->Nz, p->lat_dims};
    OCTCHK(dev_alloc(p, &p->tvwork, tv_work_elems(pg)));
    HIPCHK(hipMemset(p->p0, 0, sizeof(float2) * p->n_img() * nd));
    HIPCHK(hipMemset(p->p1, 0, sizeof(float2) * p->n_img() * nd));
  }
  if (p->hs && p->full && !p->yhat) {
    OCTCHK(dev_alloc(p, &p->yhat, w_elems(p->g)));
    HIPCHK(hipMemset(p->yhat, 0, sizeof(float2) * w_elems(p->g)));
  }
  if (pen == OCT_PEN_DTCWT && !p->dtwork) {
    ProxGeom pg{(int)p->B, (int)p->Ny, (int)p->Nx, (int)p->Nz, p->lat_dims};
    OCTCHK(dev_alloc(p, &p->dtwork, dtcwt_work_elems(pg)));
  }
  if (iters > p->hist_cap) {
    OCTCHK(dev_alloc(p, &p->hist, (size_t)iters));
    p->hist_cap = iters;
  }
  // first use: the null-stream clears above finish before the caller's stream runs
  if (p->allocs.size() != n0) HIPCHK(hipStreamSynchronize(nullptr));
  return OCT_OK;
}

std::vector<float> fgp_momenta(int n) {
  std::vector<float> mu(n);
  double t = 1.0;
  for (int k = 0; k < n; ++k) {
    const double tn = (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
    mu[k] = (float)((t - 1.0) / tn);
    t = tn;
  }
  return mu;
}

ProxGeom prox_geom(const oct_plan* p) {
  return ProxGeom{(int)p->B, (int)p->Ny, (int)p->Nx, (int)p->Nz, p->lat_dims};
}

oct_status check_haar(const oct_plan* p, int levels) {
  if (levels < 1 || levels > (p->lat_dims == 1 ? 5 : 4))
    return fail(OCT_E_UNSUPPORTED, "haar_levels must be 1..5 (B-scan) or 1..4 (volume)");
  const int64_t bs = (int64_t)1 << levels;
  if (p->Nz % bs || p->Nx % bs || (p->lat_dims == 2 && p->Ny % bs))
    return fail(OCT_E_UNSUPPORTED, "Haar needs every image dimension divisible by 2^levels");
  return OCT_OK;
}

// Modulus bound of the constraint set C of eq. (16): > 0 and finite selects
// C = {|x_i| <= bound}; 0, negative or +inf select C = C^N (+inf on the device).
oct_status check_bound(double b) {
  if (std::isnan(b)) return fail(OCT_E_INVALID, "bound is NaN");
  return OCT_OK;
}
float bound_f(double b) { return (b > 0 && std::isfinite(b)) ? (float)b : INFINITY; }

oct_status check_dtcwt(const oct_plan* p, int levels) {
  if (levels < 1 || levels > (p->lat_dims == 1 ? 5 : 4))
    return fail(OCT_E_UNSUPPORTED, "DT-CWT levels must be 1..5 (B-scan) or 1..4 (volume)");
  const int64_t bs = (int64_t)1 << levels;
  if (p->Nz % bs || p->Nx % bs || (p->lat_dims == 2 && p->Ny % bs))
    return fail(OCT_E_UNSUPPORTED, "the DT-CWT needs every image dimension divisible by 2^levels");
  return OCT_OK;
}

// z = prox(v) with FP64 partials of R(z) in p->partial[0..*np) (for the DT-CWT
// only when want_value: R(z) then needs a transform of z of its own)
oct_status run_prox(oct_plan* p, int pen, float tau, float bound, int tv_inner, int haar_levels, const float2* v,
                    float2* z, const float2* p_in, float2* p_out, int* np, hipStream_t s, bool want_value = false) {
  ProxGeom pg = prox_geom(p);
  if (pen == OCT_PEN_L1) {
    const int nb = 1024;
    HIPCHK(launch_prox_l1(v, z, p->n_img(), tau, bound, p->partial, nb, s));
    *np = nb;
  } else if (pen == OCT_PEN_HAAR) {
    if (bound < INFINITY) return fail(OCT_E_UNSUPPORTED, "a modulus bound with the Haar prox has no closed form");
    OCTCHK(check_haar(p, haar_levels));
    // |detail| partials only when the value is wanted (the kernel skips them otherwise)
    HIPCHK(launch_prox_haar(pg, haar_levels, v, z, tau, want_value ? p->partial : nullptr, s));
    *np = want_value ? haar_partials(pg, haar_levels) : 0;
  } else if (pen == OCT_PEN_TV) {
    if (tv_inner < 1 || tv_inner > 1000) return fail(OCT_E_INVALID, "tv_inner must be 1..1000");
    std::vector<float> mom = fgp_momenta(tv_inner);
    // TV(z) partials only when the value is wanted (the kernels skip it otherwise)
    HIPCHK(launch_prox_tv(pg, tv_inner, mom.data(), v, z, p_in, p_out, tau, bound,
                          want_value ? p->partial : nullptr, p->tvwork, s));
    *np = want_value ? tv_partials(pg, tv_inner) : 0;
  } else if (pen == OCT_PEN_DTCWT) {
    if (bound < INFINITY) return fail(OCT_E_UNSUPPORTED, "a modulus bound with the DT-CWT step has no closed form");
    OCTCHK(check_dtcwt(p, haar_levels));
    HIPCHK(launch_prox_dtcwt(pg, haar_levels, v, z, tau, p->dtwork, s));
    *np = 1;
    if (want_value) {
      HIPCHK(launch_dtcwt_value(pg, haar_levels, z, p->dtwork, p->partial, s));
      *np = dtcwt_partials(pg, haar_levels);
    } else {
      HIPCHK(launch_zero(reinterpret_cast<float2*>(p->partial), 1, s));
    }
  } else {
    return fail(OCT_E_INVALID, "unknown penalty");
  }
  return OCT_OK;
}

}  // namespace

extern "C" {

const char* oct_last_error(void) { return g_err.c_str(); }


size_t oct_plan_footprint_bytes(const oct_geometry* g, int32_t penalty) {
  if (validate(g) != OCT_OK) return 0;
  const int64_t Nlat = g->n_x * g->n_y;
  const int64_t N = g->batch * Nlat * g->n_depth;
  const int64_t M = g->batch * Nlat * g->n_k;
  const int64_t K = (int64_t)std::llround(g->oversamp * (double)g->n_depth);
  const int nd = g->lateral_dims + 1;
  size_t b = 0;
  b += (size_t)(K + g->n_x + g->n_y) * 8 + (size_t)g->n_depth * 4 + (size_t)g->n_k * (8 + 8) +
       (size_t)Nlat * (8 + 4) * 2 + (size_t)g->n_k * 8 + (size_t)Nlat * ((g->n_k + 31) / 32) * 4;
  b += (size_t)x1_elems(*g) * 8 + (size_t)w_elems(*g) * 8;  // workspace X1, W
  b += (size_t)Nlat * 16;                        // column-pair table of the half-spectrum path
  b += (size_t)M * 4;                            // measurements scaled per item (per-item weights)
  b += (size_t)w_elems(*g) * 8;                  // lateral spectrum of y (solves of a fully observed plan)
  if (g->model == OCT_MODEL_LITERAL)             // K's samples and the literal chain's tables
    b += (size_t)N * 8 + (size_t)g->n_depth * 16 + (size_t)g->n_k * 16;
  b += (size_t)N * 8 * 3;                        // FISTA iterates and the extrapolated point
  const bool all = penalty < 0;                  // every penalty's state and every optional buffer
  if (penalty == OCT_PEN_TV || all) b += (size_t)N * 8 * (2 * nd + 1 + nd);
  if (penalty == OCT_PEN_DTCWT || all) b += (size_t)N * 8 * (g->lateral_dims == 2 ? 24 : 8);
  if (all) b += (size_t)M * 4;                   // filled spectra / real residual (interpolated ISAM, paper backward)
  b += 64 * 1024 * 8;                            // partials, scalars, history
  return b;
}

oct_status oct_plan_create(const oct_geometry* g, const uint8_t* mask, oct_plan_t* out) {
  if (!out) return fail(OCT_E_INVALID, "out is NULL");
  *out = nullptr;
  OCTCHK(validate(g));
  OCTCHK(unsupported_sizes(g));
  int device = 0;
  HIPCHK(hipGetDevice(&device));   // before the plan exists: nothing to free on failure
  oct_plan* p = new (std::nothrow) oct_plan();
  if (!p) return fail(OCT_E_NOMEM, "host allocation failed");
  p->g = *g;
  p->device = device;
  keep_pool_memory(p->device);
  p->lat_dims = g->lateral_dims;
  p->Nz = g->n_depth;
  p->Nx = g->n_x;
  p->Ny = g->n_y;
  p->Mk = g->n_k;
  p->B = g->batch;
  p->Nlat = p->Nx * p->Ny;
  p->K = (int64_t)std::llround(g->oversamp * (double)g->n_depth);
  p->nc = (int)(p->Nz / 2);
  p->J = g->kb_width;
  p->dk = (g->k_max - g->k_min) / (double)(p->Mk - 1);
  p->dz = g->dz > 0 ? g->dz : kPi / (2.0 * (double)p->Nz * p->dk);
  p->zf = g->z_focus >= 0 ? g->z_focus : p->nc * p->dz;
  const double s = g->oversamp;
  p->kbb = g->kb_beta > 0 ? g->kb_beta
                          : kPi * std::sqrt((double)p->J * p->J / (s * s) * (s - 0.5) * (s - 0.5) - 0.8);
  p->ct = (double)p->K * p->dz / (2.0 * kPi);
  p->df = p->zf - p->nc * p->dz;
  if (std::fabs(p->df) < 1e-12 * std::max(1.0, std::fabs(p->zf))) p->df = 0.0;
  factorize((int)p->K, p->fK);
  factorize((int)p->Nx, p->fX);
  factorize((int)p->Ny, p->fY);

  oct_status st = OCT_OK;
  auto cleanup = [&](oct_status e) {
    oct_plan_destroy(p);
    return e;
  };
  // wavenumber grid as linspace(k_min, k_max, M_k) with an exact last point
  std::vector<double> k(p->Mk), k2x4(p->Mk);
  for (int64_t m = 0; m < p->Mk; ++m) k[m] = g->k_min + (double)m * p->dk;
  k[p->Mk - 1] = g->k_max;
  std::vector<float2> ph(p->Mk);
  const double mc = (double)(p->Mk - 1) / 2.0;
  for (int64_t m = 0; m < p->Mk; ++m) {
    k2x4[m] = 4.0 * k[m] * k[m];
    const double u = (double)m - mc;
    const double om = g->disp_a * u * u + g->disp_b * u * u * u;
    const double a = -2.0 * k[m] * p->zf + om;
    ph[m] = make_float2((float)std::cos(a), (float)std::sin(a));
  }
  std::vector<float2> ph_nd(p->Mk);
  for (int64_t m = 0; m < p->Mk; ++m) {
    const double a = -2.0 * k[m] * p->zf;
    ph_nd[m] = make_float2((float)std::cos(a), (float)std::sin(a));
  }
  std::vector<double> q2(p->Nlat);
  std::vector<float> beam(p->Nlat);
  auto fftfreq = [](int64_t i, int64_t n, double d) {
    const int64_t h = (n - 1) / 2 + 1;
    const double f = (i < h) ? (double)i : (double)(i - n);
    return f / ((double)n * d);
  };
  for (int64_t iy = 0; iy < p->Ny; ++iy) {
    for (int64_t ix = 0; ix < p->Nx; ++ix) {
      const double qx = 2.0 * kPi * fftfreq(ix, p->Nx, g->dx);
      const double qy = (p->lat_dims == 2) ? 2.0 * kPi * fftfreq(iy, p->Ny, g->dy) : 0.0;
      const double qq = qy * qy + qx * qx;
      q2[iy * p->Nx + ix] = qq;
      beam[iy * p->Nx + ix] = g->beam_waist > 0 ? (float)std::exp(-qq * g->beam_waist * g->beam_waist / 8.0) : 1.f;
    }
  }
  std::vector<float> deap(p->Nz);
  for (int64_t n = 0; n < p->Nz; ++n) {
    const double f = (double)(n - p->nc) / (double)p->K;
    deap[n] = (float)(1.0 / kb0_ft(f, p->J, p->kbb));
  }
  std::vector<float> kbc;
  kb_pieces(p->J, p->kbb, kbc);
  if ((st = upload(p, &p->twK, twiddles(p->fK))) != OCT_OK) return cleanup(st);
  if ((st = upload(p, &p->twX, twiddles(p->fX))) != OCT_OK) return cleanup(st);
  if ((st = upload(p, &p->twY, twiddles(p->fY))) != OCT_OK) return cleanup(st);
  if ((st = upload(p, &p->k2x4, k2x4)) != OCT_OK) return cleanup(st);
  if ((st = upload(p, &p->phase, ph)) != OCT_OK) return cleanup(st);
  if ((st = upload(p, &p->q2, q2)) != OCT_OK) return cleanup(st);
  if ((st = upload(p, &p->beam, beam)) != OCT_OK) return cleanup(st);
  if ((st = upload(p, &p->deap, deap)) != OCT_OK) return cleanup(st);
  if ((st = upload(p, &p->kbc, kbc)) != OCT_OK) return cleanup(st);
  if ((st = upload(p, &p->phase_nd, ph_nd)) != OCT_OK) return cleanup(st);
  if ((st = upload(p, &p->q2zero, std::vector<double>(p->Nlat, 0.0))) != OCT_OK) return cleanup(st);
  if ((st = upload(p, &p->beamone, std::vector<float>(p->Nlat, 1.f))) != OCT_OK) return cleanup(st);
  p->model = g->model;
  if (p->model == OCT_MODEL_LITERAL) {
    // K at the even detector wavenumbers (same grid formula as k above), the
    // N-point and 2N-point transforms, e^{j Omega} of all pixels
    std::vector<double> k2e(p->Nz);
    std::vector<float2> phe(p->Nz), om(p->Mk);
    for (int64_t j = 0; j < p->Nz; ++j) {
      const double kj = k[2 * j];
      k2e[j] = 4.0 * kj * kj;
      const double a = -2.0 * kj * p->zf;
      phe[j] = make_float2((float)std::cos(a), (float)std::sin(a));
    }
    for (int64_t m = 0; m < p->Mk; ++m) {
      const double u = (double)m - mc;
      const double o = g->disp_a * u * u + g->disp_b * u * u * u;
      om[m] = make_float2((float)std::cos(o), (float)std::sin(o));
    }
    factorize((int)p->Nz, p->fN);
    if ((st = upload(p, &p->twN, twiddles(p->fN))) != OCT_OK) return cleanup(st);
    if ((st = upload(p, &p->k2x4e, k2e)) != OCT_OK) return cleanup(st);
    if ((st = upload(p, &p->phase_e, phe)) != OCT_OK) return cleanup(st);
    if ((st = upload(p, &p->omph, om)) != OCT_OK) return cleanup(st);
    if ((st = ensure_analytic(p)) != OCT_OK) return cleanup(st);
    if ((st = dev_alloc(p, &p->Wn, p->n_img())) != OCT_OK) return cleanup(st);
  }

  if (mask) {
    p->mask_words = (int)((p->Mk + 31) / 32);
    std::vector<uint32_t> bits((size_t)p->Nlat * p->mask_words, 0u);
    for (int64_t l = 0; l < p->Nlat; ++l)
      for (int64_t m = 0; m < p->Mk; ++m) {
        if (mask[l * p->Mk + m]) bits[(size_t)l * p->mask_words + (m >> 5)] |= 1u << (m & 31);
        else p->full = false;
      }
    if ((st = upload(p, &p->mask, bits)) != OCT_OK) return cleanup(st);
  }
  // column pairs (q, -q) of the half-spectrum path: q is canonical when
  // q_x != -q_x (mod n_x) and q_x <= n_x / 2, or q_x = -q_x and q_y <= -q_y
  // (mod n_y); a pair writes the half-spectrum slot of q and, when -q has a
  // slot too (q_x = -q_x, q_y != -q_y), that one
  p->Nxh = p->Nx / 2 + 1;
  // rows of the half spectrum keep the full n_x stride (W is full-size): with
  // the packed n_x / 2 + 1 stride the volume's y passes and residual seam ran
  // 20% slower per byte (1.37 vs 1.13 ms per seam at 2048 x 256 x 256).  A
  // volume pads it by one slot: with a power-of-two n_x the y stride n_x n_k
  // is a power of two, and the half-spectrum y passes ran 8% slower for it
  // (seam 1.065 vs 0.976 ms at 2048 x 256 x 256).
  p->Nxs = w_slot_stride(p->g);
  // X1 pads its y rows the same way (its y passes have the same stride problem)
  p->X1s = w_slot_stride(p->g);
  if (p->model == OCT_MODEL_DIRECT) {
    std::vector<int4> pr;
    for (int64_t iy = 0; iy < p->Ny; ++iy) {
      for (int64_t ix = 0; ix < p->Nxh; ++ix) {
        const int64_t jx = (p->Nx - ix) % p->Nx, jy = (p->Ny - iy) % p->Ny;
        const bool xself = jx == ix;
        if (xself && iy > jy) continue;   // the partner of a canonical column
        int4 e;
        e.x = (int)(iy * p->Nx + ix);
        e.y = (int)(jy * p->Nx + jx);
        e.z = (int)(iy * p->Nxs + ix);
        e.w = (xself && jy != iy) ? (int)(jy * p->Nxs + ix) : -1;
        pr.push_back(e);
      }
    }
    p->n_pairs = (int)pr.size();
    if ((st = upload(p, &p->pairs, pr)) != OCT_OK) return cleanup(st);
    p->hs = nufft_pair_supported(nufft_args(p));
  }
  if ((st = dev_alloc(p, &p->X1, x1_elems(p->g))) != OCT_OK) return cleanup(st);
  if ((st = dev_alloc(p, &p->W, w_elems(p->g))) != OCT_OK) return cleanup(st);
  if (hipMemset(p->X1, 0, sizeof(float2) * x1_elems(p->g)) != hipSuccess ||
      hipMemset(p->W, 0, sizeof(float2) * w_elems(p->g)) != hipSuccess ||
      hipStreamSynchronize(nullptr) != hipSuccess)
    return cleanup(fail(OCT_E_DEVICE, "hipMemset of the workspace failed"));
  p->partial_cap = partial_need(p);
  if ((st = dev_alloc(p, &p->partial, (size_t)p->partial_cap * 2)) != OCT_OK) return cleanup(st);
  if ((st = dev_alloc(p, &p->dscal, 16)) != OCT_OK) return cleanup(st);
  // the adjoint column kernel may need more than 64 KB of dynamic LDS
  *out = p;
  return OCT_OK;
}

oct_status oct_plan_destroy(oct_plan_t p) {
  if (!p) return OCT_OK;
  hipDeviceSynchronize();
  for (void* a : p->allocs) hipFreeAsync(a, nullptr);
  hipStreamSynchronize(nullptr);
  delete p;
  return OCT_OK;
}

oct_status oct_plan_release(oct_plan_t p) {
  if (!p) return OCT_OK;
  int cur = 0;
  hipGetDevice(&cur);
  if (cur != p->device) hipSetDevice(p->device);
  for (void* a : p->allocs) hipFreeAsync(a, nullptr);   // ordered on the null stream, no device-wide wait
  if (cur != p->device) hipSetDevice(cur);
  delete p;
  return OCT_OK;
}

oct_status oct_forward(oct_plan_t p, const void* x, float* y, void* stream) {
  if (!p || !x || !y) return fail(OCT_E_INVALID, "null argument");
  hipStream_t s = S(stream);
  OCTCHK(run_lat_forward(p, (const float2*)x, nullptr, nullptr, 0.f, s));
  OCTCHK(run_cols_fwd(p, s, p->hs));
  OCTCHK(run_meas_forward(p, y, s, p->hs));
  return OCT_OK;
}

oct_status oct_adjoint(oct_plan_t p, const float* r, void* x, void* stream) {
  if (!p || !r || !x) return fail(OCT_E_INVALID, "null argument");
  hipStream_t s = S(stream);
  OCTCHK(run_meas_adjoint(p, r, s, p->hs));
  OCTCHK(run_cols_adj(p, s, p->hs));
  OCTCHK(run_lat_adjoint(p, (float2*)x, s));
  return OCT_OK;
}

oct_status oct_adjoint_paper(oct_plan_t p, const float* r, void* x, void* stream) {
  if (!p || !r || !x) return fail(OCT_E_INVALID, "null argument");
  hipStream_t s = S(stream);
  OCTCHK(run_meas_backward_paper(p, r, s));
  OCTCHK(run_cols_adj(p, s, false));
  OCTCHK(run_lat_adjoint(p, (float2*)x, s));
  return OCT_OK;
}

oct_status oct_direct(oct_plan_t p, int32_t kind, const float* y, void* x, void* stream) {
  if (!p || !y || !x) return fail(OCT_E_INVALID, "null argument");
  hipStream_t s = S(stream);
  switch (kind) {
    case OCT_DIRECT_AXIAL:
    case OCT_DIRECT_DISPERSION: {
      // every A-scan as the lateral-frequency-zero column; no lateral transforms
      HIPCHK(launch_meas_to_complex(y, p->mask, p->mask_words, (int)p->Mk, (int)p->Nlat, p->n_meas(), p->W, s));
      NufftArgs a = nufft_args(p);
      a.q2 = p->q2zero;
      a.beam = p->beamone;
      a.phase = (kind == OCT_DIRECT_AXIAL) ? p->phase_nd : p->phase;
      a.xs = (int)p->Nx;   // the caller's image: dense rows
      HIPCHK(launch_nufft_adj(a, p->W, (float2*)x, s));
      return OCT_OK;
    }
    case OCT_DIRECT_ISAM:
      return oct_adjoint(p, y, x, stream);
    case OCT_DIRECT_INTERP_ISAM: {
      if (!p->yfill) OCTCHK(dev_alloc(p, &p->yfill, (size_t)p->n_meas()));
      HIPCHK(launch_interp_fill(y, p->mask, p->mask_words, (int)p->Mk, (int)p->Nlat, p->B * p->Nlat, p->yfill, s));
      OCTCHK(run_meas_adjoint(p, p->yfill, s, p->hs, false));
      OCTCHK(run_cols_adj(p, s, p->hs));
      return run_lat_adjoint(p, (float2*)x, s);
    }
    default:
      return fail(OCT_E_INVALID, "unknown direct reconstruction kind");
  }
}

oct_status oct_ncc(oct_plan_t p, const void* x, const void* z, double* r_out, void* stream) {
  if (!p || !x || !z || !r_out) return fail(OCT_E_INVALID, "null argument");
  hipStream_t s = S(stream);
  const int64_t n = p->n_img();
  const int nb = ncc_blocks(n, 2 * p->partial_cap);
  HIPCHK(launch_ncc_sums((const float2*)x, (const float2*)z, n, p->partial, nb, p->dscal, s));
  double h[5];
  HIPCHK(hipMemcpyAsync(h, p->dscal, sizeof(h), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  const double sxz = h[2], sxx = h[3], szz = h[4];
  if (!(sxx > 0.0) || !(szz > 0.0)) return fail(OCT_E_INVALID, "an image has constant magnitude: NCC undefined");
  *r_out = sxz / (std::sqrt(sxx) * std::sqrt(szz));
  return OCT_OK;
}

oct_status oct_ncc_noalloc(const void* x, const void* z, int64_t n, double* r_out, void* stream) {
  if (!x || !z || !r_out) return fail(OCT_E_INVALID, "null argument");
  if (n < 1 || n > OCT_NCC_NOALLOC_MAX_N) return fail(OCT_E_INVALID, "n must be in 1..2^40");
  // same block count as oct_ncc (its plan-held partial buffer never caps it
  // below NCC_NOALLOC_MAX_BLOCKS), so the sums run in the same order
  const int nb = ncc_blocks(n, 3 * NCC_NOALLOC_MAX_BLOCKS);
  if (3 * nb + 5 > NCC_NOALLOC_SCRATCH_DOUBLES) return fail(OCT_E_INVALID, "internal: NCC partials exceed the scratch");
  double* scr = nullptr;
  HIPCHK(ncc_noalloc_scratch(&scr));
  hipStream_t s = S(stream);
  double* dsc = scr + 3 * NCC_NOALLOC_MAX_BLOCKS;
  HIPCHK(launch_ncc_sums((const float2*)x, (const float2*)z, n, scr, nb, dsc, s));
  HIPCHK(launch_ncc_finish(dsc, r_out, s));
  return OCT_OK;
}

oct_status oct_grad(oct_plan_t p, const void* x, const float* y, void* gout, double* half_resid_sq, void* stream) {
  if (!p || !x || !y || !gout) return fail(OCT_E_INVALID, "null argument");
  hipStream_t s = S(stream);
  int np = 0;
  // residual partials only when the caller asks for 1/2 ||r||^2.  Per call,
  // Y_h costs a lateral pass over y: a win for a volume, whose general seam
  // takes three passes (y, x, y), and where the one-kernel column pair saves
  // the spectrum's round trip; a B-scan whose pairs need the two kernels
  // keeps its single seam pass.
  if (spectral_seam(p, false) && (p->lat_dims == 2 || nufft_normal_pair_supported(nufft_args(p)))) {
    OCTCHK(run_meas_adjoint(p, y, s, true));   // W = Y_h, read by the column kernels
    OCTCHK(run_lat_forward(p, (const float2*)x, nullptr, nullptr, 0.f, s));
    OCTCHK(run_cols_normal(p, p->W, half_resid_sq ? p->partial : nullptr, &np, s));
    if (half_resid_sq) HIPCHK(launch_reduce_sum(p->partial, np, half_resid_sq, 0.5, 0, s));
    OCTCHK(run_lat_adjoint(p, (float2*)gout, s));
    return OCT_OK;
  } else {
    OCTCHK(run_lat_forward(p, (const float2*)x, nullptr, nullptr, 0.f, s));
    OCTCHK(run_cols_fwd(p, s, p->hs));
    OCTCHK(run_normal(p, y, half_resid_sq ? p->partial : nullptr, &np, s, p->hs));
  }
  if (half_resid_sq) HIPCHK(launch_reduce_sum(p->partial, np, half_resid_sq, 0.5, 0, s));
  OCTCHK(run_cols_adj(p, s, p->hs));
  OCTCHK(run_lat_adjoint(p, (float2*)gout, s));
  return OCT_OK;
}

oct_status oct_prox(oct_plan_t p, int32_t pen, double lambda, double delta, int32_t tv_inner, int32_t haar_levels,
                    double bound, const void* v, void* z, void* state, void* stream) {
  if (!p || !v || !z) return fail(OCT_E_INVALID, "null argument");
  if (v == z) return fail(OCT_E_INVALID, "v and z may not alias");
  if (!(lambda >= 0) || !(delta > 0)) return fail(OCT_E_INVALID, "need lambda >= 0 and delta > 0");
  OCTCHK(check_bound(bound));
  hipStream_t s = S(stream);
  OCTCHK(ensure_solver_state(p, pen, 1));
  const float tau = (float)(lambda * delta);
  const float bf = bound_f(bound);
  int np = 0;
  if (pen == OCT_PEN_TV) {
    if (!(tau > 0)) {
      // no TV term: z = P_C(v)
      if (bf < INFINITY) HIPCHK(launch_prox_l1((const float2*)v, (float2*)z, p->n_img(), 0.f, bf, p->partial, 1024, s));
      else HIPCHK(launch_copy((const float2*)v, (float2*)z, p->n_img(), s));
      return OCT_OK;
    }
    const int64_t npel = p->n_img() * (p->lat_dims + 1);
    OCTCHK(run_prox(p, pen, tau, bf, tv_inner, haar_levels, (const float2*)v, (float2*)z, (const float2*)state,
                    p->p0, &np, s));
    if (state) HIPCHK(launch_copy(p->p0, (float2*)state, npel, s));
    return OCT_OK;
  }
  return run_prox(p, pen, tau, bf, tv_inner, haar_levels, (const float2*)v, (float2*)z, nullptr, nullptr, &np, s);
}

oct_status oct_dtcwt_filter(int32_t which, float* h0, int32_t* n) {
  if (!h0 || !n) return fail(OCT_E_INVALID, "null argument");
  if (which < 0 || which > 3) return fail(OCT_E_INVALID, "which must be 0..3");
  int m = 0;
  dtcwt_filter_taps(which, h0, &m);
  *n = m;
  return OCT_OK;
}

oct_status oct_lipschitz(oct_plan_t p, int32_t iters, uint64_t seed, int32_t flags, double* L_out, void* stream) {
  if (!p || !L_out || iters < 1) return fail(OCT_E_INVALID, "bad argument");
  if (flags & ~(int32_t)OCT_SOLVE_PAPER_BACKWARD) return fail(OCT_E_INVALID, "unknown flags");
  const bool paper = (flags & OCT_SOLVE_PAPER_BACKWARD) != 0;
  hipStream_t s = S(stream);
  OCTCHK(ensure_solver_state(p, OCT_PEN_L1, 1));
  if (paper) OCTCHK(ensure_analytic(p));
  const int64_t n = p->n_img();
  const int nb = 1024;
  HIPCHK(launch_fill_counter_uniform(p->za, n, seed, s));
  HIPCHK(launch_norm2_partial(p->za, n, p->partial, nb, s));
  HIPCHK(launch_reduce_sum(p->partial, nb, p->dscal, 1.0, 0, s));
  HIPCHK(launch_scale_by_inv_sqrt(p->za, p->za, n, p->dscal, s));
  for (int it = 0; it < iters; ++it) {
    OCTCHK(run_lat_forward(p, p->za, nullptr, nullptr, 0.f, s));
    if (spectral_seam(p, paper)) {
      OCTCHK(run_cols_normal(p, nullptr, nullptr, nullptr, s));
    } else {
      OCTCHK(run_cols_fwd(p, s, p->hs && !paper));
      if (paper) OCTCHK(run_normal_paper(p, nullptr, nullptr, nullptr, s));
      else OCTCHK(run_normal(p, nullptr, nullptr, nullptr, s, p->hs));
      OCTCHK(run_cols_adj(p, s, p->hs && !paper));
    }
    OCTCHK(run_lat_adjoint(p, p->zb, s));
    HIPCHK(launch_norm2_partial(p->zb, n, p->partial, nb, s));
    HIPCHK(launch_reduce_sum(p->partial, nb, p->dscal, 1.0, 0, s));
    HIPCHK(launch_scale_by_inv_sqrt(p->zb, p->za, n, p->dscal, s));
  }
  double sumsq = 0.0;
  HIPCHK(hipMemcpyAsync(&sumsq, p->dscal, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  *L_out = std::sqrt(sumsq);
  return OCT_OK;
}

oct_status oct_mbir_solve(oct_plan_t p, const float* y, const oct_solve_params* prm, void* x_out,
                          oct_solve_report* rep, void* stream) {
  if (!p || !y || !prm || !x_out) return fail(OCT_E_INVALID, "null argument");
  if (prm->iters < 1) return fail(OCT_E_INVALID, "iters must be >= 1");
  if (prm->k0 < 0 || prm->k0 > (1 << 24)) return fail(OCT_E_INVALID, "k0 must be in 0..2^24");
  if (prm->k0 > 0 && !prm->x0) return fail(OCT_E_INVALID, "a resumed solve (k0 > 0) needs x0 = z^k0");
  if (prm->z_prev0 && !prm->x0) return fail(OCT_E_INVALID, "z_prev0 needs x0");
  if (prm->penalty < 0 || prm->penalty > 3) return fail(OCT_E_INVALID, "unknown penalty");
  if (prm->penalty == OCT_PEN_DTCWT) OCTCHK(check_dtcwt(p, prm->haar_levels));
  if (!(prm->lambda >= 0)) return fail(OCT_E_INVALID, "lambda must be >= 0");
  if (prm->penalty == OCT_PEN_HAAR) OCTCHK(check_haar(p, prm->haar_levels));
  if (prm->penalty == OCT_PEN_TV && (prm->tv_inner < 1 || prm->tv_inner > 1000))
    return fail(OCT_E_INVALID, "tv_inner must be 1..1000");
  if (prm->flags & ~(int32_t)OCT_SOLVE_PAPER_BACKWARD) return fail(OCT_E_INVALID, "unknown solve flags");
  OCTCHK(check_bound(prm->bound));
  const float bf = bound_f(prm->bound);
  if ((prm->penalty == OCT_PEN_HAAR || prm->penalty == OCT_PEN_DTCWT) && bf < INFINITY)
    return fail(OCT_E_UNSUPPORTED, "a modulus bound with the Haar or DT-CWT step has no closed form");
  const bool paper = (prm->flags & OCT_SOLVE_PAPER_BACKWARD) != 0;
  // per-item weights: every item runs at lambda = max_b lambda_b on its
  // measurement scaled by lambda / lambda_b, and its z^K is scaled back
  const bool per_item = prm->lambda_item != nullptr;
  double lambda = prm->lambda;
  ItemScales y_scale{}, z_scale{};
  if (per_item) {
    if (p->B > OCT_MAX_LAMBDA_ITEMS) return fail(OCT_E_UNSUPPORTED, "per-item weights need batch <= 64");
    if (bf < INFINITY) return fail(OCT_E_UNSUPPORTED, "per-item weights with a modulus bound");
    if (rep && rep->objective) return fail(OCT_E_UNSUPPORTED, "per-item weights with an objective report");
    if (prm->x0 || prm->z_prev_out) return fail(OCT_E_UNSUPPORTED, "per-item weights with a start point or z_prev_out");
    lambda = 0.0;
    for (int64_t b = 0; b < p->B; ++b) {
      const double l = prm->lambda_item[b];
      if (!(l > 0) || !std::isfinite(l)) return fail(OCT_E_INVALID, "per-item weights must be finite and > 0");
      lambda = std::max(lambda, l);
    }
    for (int64_t b = 0; b < p->B; ++b) {
      y_scale.s[b] = (float)(lambda / prm->lambda_item[b]);
      z_scale.s[b] = (float)(prm->lambda_item[b] / lambda);
    }
  }
  hipStream_t s = S(stream);
  OCTCHK(ensure_solver_state(p, prm->penalty, prm->iters));
  if (per_item) {
    if (!p->yitem) OCTCHK(dev_alloc(p, &p->yitem, (size_t)p->n_meas()));
    HIPCHK(launch_scale_items(y, p->yitem, p->Nlat * p->Mk, (int)p->B, y_scale, s));
    y = p->yitem;
  }
  double delta = prm->delta, Lest = 0.0;
  if (!(delta > 0)) {
    if (prm->power_iters < 1) return fail(OCT_E_INVALID, "power_iters must be >= 1 when delta <= 0");
    OCTCHK(oct_lipschitz(p, prm->power_iters, prm->seed, prm->flags, &Lest, stream));
    // L = 0: nothing observed, the data term is constant and any step is admissible
    delta = Lest > 0.0 ? 1.0 / (1.05 * Lest) : 1.0;
  }
  const int64_t n = p->n_img();
  // FISTA momenta mu_k = (t_k - 1) / t_{k+1}, t_1 = 1 (FP64)
  // FISTA momenta mu_k = (t_k - 1) / t_{k+1}, t_1 = 1 (FP64), continued from
  // iteration k0 when the solve resumes
  const int k0 = prm->k0;
  std::vector<double> mu((size_t)k0 + prm->iters);
  {
    double t = 1.0;
    for (size_t k = 0; k < mu.size(); ++k) {
      const double tn = (1.0 + std::sqrt(1.0 + 4.0 * t * t)) / 2.0;
      mu[k] = (t - 1.0) / tn;
      t = tn;
    }
  }
  float2* zc = p->za;   // z^{k-1}
  float2* zo = p->zb;   // z^{k-2}
  if (prm->x0) {
    HIPCHK(launch_copy((const float2*)prm->x0, zc, n, s));
    HIPCHK(launch_copy((const float2*)(prm->z_prev0 ? prm->z_prev0 : prm->x0), zo, n, s));
  } else {
    HIPCHK(launch_zero(zc, n, s));
    HIPCHK(launch_zero(zo, n, s));
  }
  const bool want_obj = rep && rep->objective;
  const float tau = (float)(lambda * delta);
  float2* pin = nullptr;
  float2* pout = p->p0;
  if (k0 > 0 && prm->penalty == OCT_PEN_TV && p->tv_last) {   // the dual where the last solve ended
    pin = p->tv_last;
    pout = (pin == p->p0) ? p->p1 : p->p0;
  }
  const bool fused_l1 = (prm->penalty == OCT_PEN_L1) && p->lat_dims == 1;
  if (paper) {
    // set up before any work: fails when n_k does not suit the analytic-signal transform
    OCTCHK(ensure_analytic(p));
    if (!p->yfill) OCTCHK(dev_alloc(p, &p->yfill, (size_t)p->n_meas()));
  }
  double* res_part = p->partial;
  double* pen_part = p->partial + p->partial_cap;
  const bool spec = spectral_seam(p, paper);
  if (spec) OCTCHK(run_meas_adjoint(p, y, s, true, true, p->yhat));   // Y_h, once per solve
  float mu_prev = k0 > 0 ? (float)mu[k0 - 1] : 0.f;
  if (fused_l1) OCTCHK(run_lat_forward(p, nullptr, zc, zo, mu_prev, s));
  for (int k = 0; k < prm->iters; ++k) {
    if (!fused_l1) OCTCHK(run_lat_forward(p, nullptr, zc, zo, mu_prev, s, p->xext));
    int nres = 0, npen = 0;
    // residual partials only for the objective
    if (spec) {
      OCTCHK(run_cols_normal(p, p->yhat, want_obj ? res_part : nullptr, &nres, s));
    } else {
      OCTCHK(run_cols_fwd(p, s, p->hs && !paper));
      if (paper) OCTCHK(run_normal_paper(p, y, want_obj ? res_part : nullptr, &nres, s));
      else OCTCHK(run_normal(p, y, want_obj ? res_part : nullptr, &nres, s, p->hs));
      OCTCHK(run_cols_adj(p, s, p->hs && !paper));
    }
    if (fused_l1) {
      LatArgs a = lat_args(p, lines_x(p, (int)p->Nz), false);
      a.src = p->X1;
      a.dst = p->X1;
      a.inverse = 1;
      a.z = zc;
      a.zo = zo;
      a.mu = mu_prev;
      a.mu_next = (float)mu[k0 + k];
      a.delta = (float)delta;
      a.tau = tau;
      a.bound = bf;
      a.partial = want_obj ? pen_part : nullptr;   // |z| partials only for the objective
      npen = lat_blocks(a);
      HIPCHK(launch_lateral(LAT_UPDATE_L1, a, s));
    } else {
      if (p->lat_dims == 2) {
        LatArgs b = lat_args(p, lines_y_x1(p, (int)p->Nz), true);
        b.src = p->X1;
        b.dst = p->X1;
        b.inverse = 1;
        HIPCHK(launch_lateral(LAT_FFT, b, s));
      }
      // v = x - delta grad overwrites x in place (same layout, each element
      // read then written by one thread); X1's rows may be padded, the image's not
      LatArgs a = lat_args(p, lines_x(p, (int)p->Nz), false);
      a.src = p->X1;
      a.sa_in = p->X1s * p->Nz;
      a.dst = p->xext;
      a.inverse = 1;
      a.z = p->xext;   // x as the forward pass formed it
      a.delta = (float)delta;
      HIPCHK(launch_lateral(LAT_UPDATE, a, s));
      // z^k -> zo (z^{k-2} is no longer needed)
      if (prm->penalty == OCT_PEN_TV && !(tau > 0)) {
        // no TV term (its partials are zero): z = P_C(v)
        if (bf < INFINITY) HIPCHK(launch_prox_l1(p->xext, zo, n, 0.f, bf, nullptr, 1024, s));
        else HIPCHK(launch_copy(p->xext, zo, n, s));
        HIPCHK(launch_zero(reinterpret_cast<float2*>(pen_part), 1, s));
        npen = 1;
      } else {
        double* save = p->partial;
        p->partial = pen_part;
        oct_status st = run_prox(p, prm->penalty, tau, bf, prm->tv_inner, prm->haar_levels, p->xext, zo, pin, pout,
                                 &npen, s, want_obj);
        p->partial = save;
        OCTCHK(st);
        if (prm->penalty == OCT_PEN_TV) {
          pin = pout;
          pout = (pout == p->p0) ? p->p1 : p->p0;
        }
      }
    }
    if (want_obj) HIPCHK(launch_objective(res_part, nres, pen_part, npen, lambda, p->hist + k, s));
    std::swap(zc, zo);
    mu_prev = (float)mu[k0 + k];
  }
  if (prm->penalty == OCT_PEN_TV) p->tv_last = pin;
  if (per_item) HIPCHK(launch_scale_items(zc, (float2*)x_out, p->Nlat * p->Nz, (int)p->B, z_scale, s));
  else HIPCHK(launch_copy(zc, (float2*)x_out, n, s));
  if (prm->z_prev_out) HIPCHK(launch_copy(zo, (float2*)prm->z_prev_out, n, s));   // z^{K-1}
  if (rep) {
    rep->delta_used = delta;
    rep->lipschitz_est = Lest;
    if (want_obj) {
      HIPCHK(hipMemcpyAsync(rep->objective, p->hist, sizeof(double) * prm->iters, hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
    }
  }
  return OCT_OK;
}

oct_status oct_run_stage(oct_plan_t p, int32_t stage, int32_t pen, const float* y, void* stream) {
  if (!p) return fail(OCT_E_INVALID, "null plan");
  if (pen < 0 || pen > 3) return fail(OCT_E_INVALID, "unknown penalty");
  hipStream_t s = S(stream);
  OCTCHK(ensure_solver_state(p, pen, 1));
  switch (stage) {
    case OCT_STAGE_LAT_FWD:
      return run_lat_forward(p, nullptr, p->za, p->zb, 0.5f, s, p->xext);
    case OCT_STAGE_NUFFT_FWD:   // as in a solve without the objective
      if (spectral_seam(p, false)) return run_cols_fwd_res(p, p->yhat, nullptr, nullptr, s);
      OCTCHK(run_cols_fwd(p, s, p->hs));
      return OCT_OK;
    case OCT_STAGE_NORMAL: {
      if (!y) return fail(OCT_E_INVALID, "OCT_STAGE_NORMAL needs y");
      int np = 0;
      return run_normal(p, y, nullptr, &np, s, p->hs);   // as in a solve without the objective
    }
    case OCT_STAGE_NUFFT_ADJ:
      OCTCHK(run_cols_adj(p, s, p->hs));
      return OCT_OK;
    case OCT_STAGE_LAT_UPDATE: {
      if (p->lat_dims == 2) {
        LatArgs b = lat_args(p, lines_y_x1(p, (int)p->Nz), true);
        b.src = p->X1;
        b.dst = p->X1;
        b.inverse = 1;
        HIPCHK(launch_lateral(LAT_FFT, b, s));
      }
      LatArgs a = lat_args(p, lines_x(p, (int)p->Nz), false);
      a.src = p->X1;
      a.sa_in = p->X1s * p->Nz;
      a.dst = p->xext;
      a.inverse = 1;
      a.z = p->xext;
      a.delta = 1e-3f;
      HIPCHK(launch_lateral(LAT_UPDATE, a, s));
      return OCT_OK;
    }
    case OCT_STAGE_NUFFT_NORMAL:
      if (!spectral_seam(p, false)) return fail(OCT_E_UNSUPPORTED, "OCT_STAGE_NUFFT_NORMAL needs a fully observed plan");
      return run_cols_normal(p, p->yhat, nullptr, nullptr, s);
    case OCT_STAGE_PROX: {
      int np = 0;
      return run_prox(p, pen, 1e-3f, INFINITY, 10, 3, p->xext, p->zb, pen == OCT_PEN_TV ? p->p0 : nullptr,
                      pen == OCT_PEN_TV ? p->p1 : nullptr, &np, s);
    }
    default:
      return fail(OCT_E_INVALID, "unknown stage");
  }
}

}  // extern "C"
