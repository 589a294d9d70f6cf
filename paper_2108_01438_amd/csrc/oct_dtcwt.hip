// Dual-tree complex wavelet transform (Sec. 2.2; the DT-CWT of Selesnick,
// Baraniuk and Kingsbury) for B-scans, and its shrinkage step.
//
// Filters (designed on the host at first use, FP64, rounded once): Selesnick's
// common-factor construction of approximate Hilbert-transform pairs,
// h = F D and g = F D~, D the degree-L maximally flat allpass denominator for
// a half-sample delay (D~(z) = z^-L D(1/z)) and F = Q (1 + 1/z)^K with Q the
// minimum-phase spectral factor of the symmetric R that makes
// (z + 2 + 1/z)^K D(z) D(1/z) R(z) halfband.  First level: the 6-tap
// Daubechies filter (K = 3, L = 0) for tree a and the same one sample later
// for tree b; later levels: the 12-tap pair (K = 3, L = 3).
//
// Transform: four separable orthonormal 2-D DWTs (depth filters of tree a
// or b x lateral filters of tree a or b), periodic extension, per level a
// depth pass then a lateral pass, bands kept in place (Mallat layout) in one
// buffer per tree.  The detail bands of the four trees combine per element
// into the six oriented complex subbands (u1, v1) = (aa - bb, ab + ba)/sqrt2,
// (u2, v2) = (aa + bb, ab - ba)/sqrt2.  With the 1/2 scaling of the trees the
// transform W is a Parseval frame; the shrinkage step W^T soft_tau(W v) is
// computed on the unscaled trees as 1/4 sum_t T_t^T(C^T soft_{2 tau}(C T v)).
#include "oct_fft.h"

#include <cmath>
#include <complex>
#include <vector>

namespace {

constexpr int DT_MAXT = 16;

struct DtFilt {
  float h0[DT_MAXT], h1[DT_MAXT];
  int n;
};

struct DtGeom {
  int B, NX, NZ;      // image [B][NX][NZ]
  int nx, nz;         // current (sub-)array at the top-left of every item
};

// Periodic one-level filter banks along one axis of the top-left nx x nz
// sub-array of every image of the batch.  Analysis: lo[i] = sum_k h0[k]
// x[(2i + k) mod n], hi[i] likewise with h1, lo to the first half of the
// axis and hi to the second.  Synthesis is its transpose (the analysis is
// orthogonal): x[m] = sum over k with m - k even of h0[k] lo[i] + h1[k] hi[i],
// i = ((m - k) mod n) / 2.  blockIdx.y selects one of up to four (source,
// filter, destination) jobs of a launch (the four trees, or the two depth
// filters of the first level); ACC makes a synthesis job add the output of
// job y + 1 (same destination), so two trees that share the next pass are
// summed on the way.

struct DtJobs {
  const float2* src[4];
  float2* dst[4];
  DtFilt f[4];
  float scale;      // applied to synthesis outputs
};

__device__ __forceinline__ void fma2(float2& acc, float w, float2 x) {
  acc.x = fmaf(w, x.x, acc.x);
  acc.y = fmaf(w, x.y, acc.y);
}

__device__ __forceinline__ void afb_line(const DtFilt& f, const float2* __restrict__ src, int64_t stride, int n,
                                         int i, float2& lo, float2& hi) {
  lo = make_float2(0.f, 0.f);
  hi = make_float2(0.f, 0.f);
  int m = 2 * i;
  for (int k = 0; k < f.n; ++k) {
    const float2 x = src[(int64_t)m * stride];
    fma2(lo, f.h0[k], x);
    fma2(hi, f.h1[k], x);
    if (++m == n) m = 0;
  }
}

__device__ __forceinline__ float2 sfb_line(const DtFilt& f, const float2* __restrict__ src, int64_t stride, int n,
                                           int m) {
  const int h = n / 2;
  float2 x = make_float2(0.f, 0.f);
  for (int k = m & 1; k < f.n; k += 2) {
    int d = m - k;
    while (d < 0) d += n;
    const int i = d >> 1;
    fma2(x, f.h0[k], src[(int64_t)i * stride]);
    fma2(x, f.h1[k], src[(int64_t)(h + i) * stride]);
  }
  return x;
}

// depth analysis: thread = (batch, lateral l < nx, i < nz/2), i fastest
__global__ void afb_depth_kernel(DtGeom g, DtJobs J) {
  const int j = blockIdx.y;
  const int h = g.nz / 2;
  const int64_t total = (int64_t)g.B * g.nx * h;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int i = (int)(t % h);
    const int64_t r = t / h;
    const int l = (int)(r % g.nx);
    const int b = (int)(r / g.nx);
    const int64_t base = ((int64_t)b * g.NX + l) * g.NZ;
    float2 lo, hi;
    afb_line(J.f[j], J.src[j] + base, 1, g.nz, i, lo, hi);
    J.dst[j][base + i] = lo;
    J.dst[j][base + h + i] = hi;
  }
}

template <bool ACC>
__global__ void sfb_depth_kernel(DtGeom g, DtJobs J) {
  const int j = blockIdx.y * (ACC ? 2 : 1);
  const int64_t total = (int64_t)g.B * g.nx * g.nz;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int m = (int)(t % g.nz);
    const int64_t r = t / g.nz;
    const int l = (int)(r % g.nx);
    const int b = (int)(r / g.nx);
    const int64_t base = ((int64_t)b * g.NX + l) * g.NZ;
    float2 x = sfb_line(J.f[j], J.src[j] + base, 1, g.nz, m);
    if (ACC) {
      const float2 y = sfb_line(J.f[j + 1], J.src[j + 1] + base, 1, g.nz, m);
      x = make_float2(x.x + y.x, x.y + y.y);
    }
    J.dst[j][base + m] = make_float2(J.scale * x.x, J.scale * x.y);
  }
}

struct Trees {
  float2* t[4];   // trees aa, ab, ba, bb
};

__device__ __forceinline__ float2 add2(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 sub2(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// Combination of the four trees at one detail position into the two complex
// coefficients (u1, v1), (u2, v2); SHRINK shrinks both by tau2 and writes the
// trees back through the inverse combination, otherwise the moduli are added
// (scaled by 1/2 for the Parseval normalisation).
template <bool SHRINK>
__device__ __forceinline__ void dt_group(float2 (&w)[4], float tau2, double& acc) {
  const float r2 = 0.70710678118654752440f;
  float2 u1 = cscale(sub2(w[0], w[3]), r2), v1 = cscale(add2(w[1], w[2]), r2);
  float2 u2 = cscale(add2(w[0], w[3]), r2), v2 = cscale(sub2(w[1], w[2]), r2);
  const float m1 = sqrtf(u1.x * u1.x + u1.y * u1.y + v1.x * v1.x + v1.y * v1.y);
  const float m2 = sqrtf(u2.x * u2.x + u2.y * u2.y + v2.x * v2.x + v2.y * v2.y);
  if (!SHRINK) {
    acc += 0.5 * ((double)m1 + (double)m2);
    return;
  }
  const float s1 = m1 > tau2 ? 1.f - tau2 / m1 : 0.f;
  const float s2 = m2 > tau2 ? 1.f - tau2 / m2 : 0.f;
  u1 = cscale(u1, s1);
  v1 = cscale(v1, s1);
  u2 = cscale(u2, s2);
  v2 = cscale(v2, s2);
  w[0] = cscale(add2(u1, u2), r2);
  w[3] = cscale(sub2(u2, u1), r2);
  w[1] = cscale(add2(v1, v2), r2);
  w[2] = cscale(sub2(v1, v2), r2);
}

// LDS-tiled lateral synthesis.  A workgroup (4 waves) owns 64 consecutive
// depth samples (one per lane) and a run of lateral output rows; it stages
// the input rows those outputs need (periodic wrap resolved while staging) in
// LDS once, so that every tap is an LDS read instead of a strided global one.
// (The analysis stays untiled: measured faster, its taps hit the caches.)
constexpr int DT_LANES = 64;

// Threads a register-window pass needs before it replaces the per-tap kernel
// (about four workgroups per CU): below that the walk along the axis leaves
// too few threads, and the per-tap kernel's rows fit the caches anyway.
constexpr int64_t DT_WINDOW_MIN_THREADS = (int64_t)1 << 18;

__device__ __forceinline__ void dt_stage(const float2* __restrict__ src, int64_t item, int NZ, int n, int base,
                                         int nrows, int n0, int nz, int rowoff, float2* __restrict__ lds) {
  for (int e = threadIdx.x; e < nrows * DT_LANES; e += blockDim.x) {
    const int r = e / DT_LANES, c = e % DT_LANES;
    int m = (base + r) % n;
    if (m < 0) m += n;
    const int nn = n0 + c;
    lds[e] = nn < nz ? src[item + (int64_t)(rowoff + m) * NZ + nn] : make_float2(0.f, 0.f);
  }
}

// Lateral analysis of all four trees at once (thread = (batch, i < nx/2,
// depth n < nz)), with the detail bands of the level handled on the spot:
// lateral-low outputs in the depth-low half are the next level's low band
// and are written as they are; every other output is a detail coefficient,
// combined across the trees and shrunk (SHRINK, then written) or summed into
// FP64 block partials (value pass: only the low band is written).
template <bool SHRINK>
__global__ void afb_lateral4_kernel(DtGeom g, DtJobs J, float tau2, double* partial) {
  __shared__ double sh[16];
  const int h = g.nx / 2, hz = g.nz / 2;
  const int64_t total = (int64_t)g.B * h * g.nz;
  double acc = 0.0;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int n = (int)(t % g.nz);
    const int64_t r = t / g.nz;
    const int i = (int)(r % h);
    const int b = (int)(r / h);
    const int64_t item = (int64_t)b * g.NX * g.NZ + n;
    float2 lo[4], hi[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) afb_line(J.f[k], J.src[k] + item, g.NZ, g.nx, i, lo[k], hi[k]);
    const int64_t olo = item + (int64_t)i * g.NZ, ohi = item + (int64_t)(h + i) * g.NZ;
    if (n >= hz) dt_group<SHRINK>(lo, tau2, acc);
    dt_group<SHRINK>(hi, tau2, acc);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if (SHRINK || n < hz) J.dst[k][olo] = lo[k];
      if (SHRINK) J.dst[k][ohi] = hi[k];
    }
  }
  if (!SHRINK) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += sh[k];
      partial[blockIdx.x] = s;
    }
  }
}

// Lateral synthesis (the transpose of the analysis along the lateral axis):
// TS output rows per workgroup; blockIdx.y picks the job (ACC: the job pair
// summed into one destination).
template <bool ACC>
__global__ void __launch_bounds__(256) sfb_lateral_tiled(DtGeom g, DtJobs J) {
  constexpr int TS = 32;
  constexpr int NS = ACC ? 2 : 1;
  constexpr int CNT = (TS + DT_MAXT) / 2 + 1;
  __shared__ float2 lo_s[NS][CNT * DT_LANES], hi_s[NS][CNT * DT_LANES];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int n0 = blockIdx.x * DT_LANES, m0 = blockIdx.z * TS;
  const int j = blockIdx.y * NS;
  const int h = g.nx / 2;
  const int B = g.B;
  for (int b = 0; b < B; ++b) {
    const int64_t item = (int64_t)b * g.NX * g.NZ;
    const int taps = NS == 2 ? max(J.f[j].n, J.f[j + 1].n) : J.f[j].n;   // rows staged for every job
    const int ibase = (m0 - taps + 1) >> 1;
    const int cnt = (m0 + TS - 1 - ((m0 - taps + 1) & ~1)) / 2 + 1;
    if (b > 0) __syncthreads();
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      dt_stage(J.src[j + q], item, g.NZ, h, ibase, cnt, n0, g.nz, 0, lo_s[q]);
      dt_stage(J.src[j + q], item, g.NZ, h, ibase, cnt, n0, g.nz, h, hi_s[q]);
    }
    __syncthreads();
    const int n = n0 + lane;
    for (int r = 0; r < TS / 4; ++r) {
      const int m = m0 + w * (TS / 4) + r;
      if (m >= g.nx || n >= g.nz) continue;
      float2 x = make_float2(0.f, 0.f);
#pragma unroll
      for (int q = 0; q < NS; ++q) {
        const DtFilt& f = J.f[j + q];
        for (int t = m & 1; t < f.n; t += 2) {
          const int row = ((m - t) >> 1) - ibase;
          fma2(x, f.h0[t], lo_s[q][row * DT_LANES + lane]);
          fma2(x, f.h1[t], hi_s[q][row * DT_LANES + lane]);
        }
      }
      J.dst[j][item + (int64_t)m * g.NZ + n] = make_float2(J.scale * x.x, J.scale * x.y);
    }
  }
}

int dt_grid(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  return (int)(b < 1 ? 1 : b);
}

// ---------------------------------------------------------------------------
// Host filter design (FP64)
// ---------------------------------------------------------------------------
std::vector<double> conv(const std::vector<double>& a, const std::vector<double>& b) {
  std::vector<double> o(a.size() + b.size() - 1, 0.0);
  for (size_t i = 0; i < a.size(); ++i)
    for (size_t j = 0; j < b.size(); ++j) o[i + j] += a[i] * b[j];
  return o;
}

double binom(int n, int k) {
  double v = 1.0;
  for (int i = 1; i <= k; ++i) v = v * (double)(n - k + i) / (double)i;
  return v;
}

// Gaussian elimination with partial pivoting (n x n, row-major), in place.
bool solve(std::vector<double>& A, std::vector<double>& b, int n) {
  for (int c = 0; c < n; ++c) {
    int p = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[p * n + c])) p = r;
    if (std::fabs(A[p * n + c]) < 1e-300) return false;
    if (p != c) {
      for (int k = 0; k < n; ++k) std::swap(A[p * n + k], A[c * n + k]);
      std::swap(b[p], b[c]);
    }
    for (int r = c + 1; r < n; ++r) {
      const double f = A[r * n + c] / A[c * n + c];
      for (int k = c; k < n; ++k) A[r * n + k] -= f * A[c * n + k];
      b[r] -= f * b[c];
    }
  }
  for (int c = n - 1; c >= 0; --c) {
    double s = b[c];
    for (int k = c + 1; k < n; ++k) s -= A[c * n + k] * b[k];
    b[c] = s / A[c * n + c];
  }
  return true;
}

// Roots of sum_i p[i] z^(deg - i) (p[0] != 0) by the Weierstrass (Durand-Kerner)
// iteration.
std::vector<std::complex<double>> roots(const std::vector<double>& p) {
  const int deg = (int)p.size() - 1;
  std::vector<std::complex<double>> z(deg);
  const std::complex<double> seed(0.4, 0.9);
  for (int i = 0; i < deg; ++i) z[i] = std::pow(seed, i);
  for (int it = 0; it < 2000; ++it) {
    double move = 0.0;
    for (int i = 0; i < deg; ++i) {
      std::complex<double> num = p[0];
      for (int k = 1; k <= deg; ++k) num = num * z[i] + p[k];
      std::complex<double> den = p[0];
      for (int j = 0; j < deg; ++j)
        if (j != i) den *= (z[i] - z[j]);
      const std::complex<double> d = num / den;
      z[i] -= d;
      move = std::max(move, std::abs(d));
    }
    if (move < 1e-15) break;
  }
  return z;
}

// Lowpass pair (h, g) of the common-factor design with K zeros at z = -1 and a
// degree-L half-sample allpass (L = 0: Daubechies, h = g).
void design_pair(int K, int L, std::vector<double>& h, std::vector<double>& g) {
  std::vector<double> d(L + 1);
  for (int n = 0; n <= L; ++n) {
    double v = (n & 1) ? -binom(L, n) : binom(L, n);
    for (int k = 0; k < n; ++k) v *= (0.5 - L + k) / (1.5 + k);
    d[n] = v;
  }
  std::vector<double> dr(d.rbegin(), d.rend());
  std::vector<double> q0 = conv(d, dr);
  for (int k = 0; k < K; ++k) q0 = conv(q0, {1.0, 2.0, 1.0});
  const int M = K + L - 1, nP = K + L + M;
  const int neq = (nP + 1) / 2;           // = M + 1
  std::vector<double> A(neq * neq), rhs(neq, 0.0);
  rhs[0] = 1.0;
  for (int i = 0; i <= M; ++i) {
    std::vector<double> r(2 * M + 1, 0.0);
    r[M + i] = 1.0;
    r[M - i] = 1.0;
    const std::vector<double> col = conv(q0, r);    // centre index nP
    for (int e = 0; e < neq; ++e) A[e * neq + i] = col[nP + 2 * e];
  }
  solve(A, rhs, neq);
  std::vector<double> f = {1.0};
  if (M > 0) {
    std::vector<double> R(2 * M + 1);
    R[M] = rhs[0];
    for (int i = 1; i <= M; ++i) R[M + i] = R[M - i] = rhs[i];
    // minimum-phase factor: the monic polynomial of the roots inside the unit circle
    std::vector<std::complex<double>> poly = {1.0};
    for (const auto& z : roots(R))
      if (std::abs(z) < 1.0) {
        std::vector<std::complex<double>> nx(poly.size() + 1, 0.0);
        for (size_t k = 0; k < poly.size(); ++k) {
          nx[k] += poly[k];
          nx[k + 1] -= poly[k] * z;
        }
        poly = nx;
      }
    f.assign(poly.size(), 0.0);
    for (size_t k = 0; k < poly.size(); ++k) f[k] = poly[k].real();
  }
  for (int k = 0; k < K; ++k) f = conv(f, {1.0, 1.0});
  h = conv(f, d);
  g = conv(f, dr);
  double s = 0.0;
  for (double v : h) s += v;
  const double sc = std::sqrt(2.0) / s;
  for (double& v : h) v *= sc;
  for (double& v : g) v *= sc;
}

DtFilt make_filt(const std::vector<double>& h) {
  DtFilt f{};
  f.n = (int)h.size();
  for (int k = 0; k < f.n; ++k) {
    f.h0[k] = (float)h[k];
    const double hk = h[f.n - 1 - k];
    f.h1[k] = (float)((k & 1) ? -hk : hk);
  }
  return f;
}

struct DtFilters {
  DtFilt first[2], later[2];
};

DtFilters design_filters() {
  DtFilters F;
  std::vector<double> d1, d1g, ha, hb;
  design_pair(3, 0, d1, d1g);
  std::vector<double> fa(d1), fb(1, 0.0);
  fa.push_back(0.0);
  fa.push_back(0.0);
  fb.insert(fb.end(), d1.begin(), d1.end());
  fb.push_back(0.0);
  design_pair(3, 3, ha, hb);
  F.first[0] = make_filt(fa);
  F.first[1] = make_filt(fb);
  F.later[0] = make_filt(ha);
  F.later[1] = make_filt(hb);
  return F;
}

// Designed once per process (the initialisation of a function-local static
// is thread safe: plans on several host threads may ask at once).
const DtFilters& filters() {
  static const DtFilters F = design_filters();
  return F;
}

// Workspace: four tree buffers then four staging buffers, one image each.
struct DtWork {
  Trees tr;
  float2* tmp[4];
};

DtWork dt_work(float2* work, int64_t n) {
  DtWork w;
  for (int t = 0; t < 4; ++t) {
    w.tr.t[t] = work + t * n;
    w.tmp[t] = work + (4 + t) * n;
  }
  return w;
}

int dt_grid_y(int64_t n, int jobs) {
  int64_t b = (n + 255) / 256;
  const int64_t cap = 4096 / jobs;
  if (b > cap) b = cap;
  return (int)(b < 1 ? 1 : b);
}

// Workgroups of the tiled lateral synthesis (32 output rows each, the batch
// looped inside).
dim3 dt_sfb_grid(const DtGeom& g, int jobs) {
  return dim3((unsigned)((g.nz + DT_LANES - 1) / DT_LANES), (unsigned)jobs, (unsigned)((g.nx + 31) / 32));
}

// Analysis of all trees (level by level) from v into the tree buffers.
// Level 1: the two depth filters once each (v -> tmp[0], tmp[1]), then the
// lateral filters of every tree from its depth tree's staging buffer.  Later
// levels: each tree's low band through tmp[t].
// mode 0: analysis with the detail bands shrunk by tau2 on the way; mode 1:
// the value pass (block partials of sum |W x| into partial, nothing but the
// low bands written).
hipError_t dt_analysis(const DtGeom& g0, int levels, const float2* v, const DtWork& w, int mode, float tau2,
                       double* partial, hipStream_t s) {
  const DtFilters& F = filters();
  DtGeom g = g0;
  for (int lev = 0; lev < levels; ++lev) {
    const DtFilt* fs = lev == 0 ? F.first : F.later;
    const int64_t nd = (int64_t)g.B * g.nx * (g.nz / 2), nl = (int64_t)g.B * (g.nx / 2) * g.nz;
    DtJobs jd{}, jl{};
    int ndj;
    if (lev == 0) {
      ndj = 2;
      for (int p = 0; p < 2; ++p) {
        jd.src[p] = v;
        jd.dst[p] = w.tmp[p];
        jd.f[p] = fs[p];
      }
    } else {
      ndj = 4;
      for (int t = 0; t < 4; ++t) {
        jd.src[t] = w.tr.t[t];
        jd.dst[t] = w.tmp[t];
        jd.f[t] = fs[t >> 1];
      }
    }
    for (int t = 0; t < 4; ++t) {
      jl.src[t] = lev == 0 ? w.tmp[t >> 1] : w.tmp[t];
      jl.dst[t] = w.tr.t[t];
      jl.f[t] = fs[t & 1];
    }
    hipLaunchKernelGGL(afb_depth_kernel, dim3(dt_grid_y(nd, ndj), ndj), dim3(256), 0, s, g, jd);
    if (mode == 0) {
      hipLaunchKernelGGL((afb_lateral4_kernel<true>), dim3(dt_grid(nl)), dim3(256), 0, s, g, jl, tau2, nullptr);
    } else {
      hipLaunchKernelGGL((afb_lateral4_kernel<false>), dim3(dt_grid(nl)), dim3(256), 0, s, g, jl, 0.f, partial);
      partial += dt_grid(nl);
    }
    g.nx /= 2;
    g.nz /= 2;
  }
  return hipGetLastError();
}



// ---------------------------------------------------------------------------
// Volumes: eight trees (depth, x, y filter trees), a pass per axis and level.
// ---------------------------------------------------------------------------
struct Dt3Geom {
  int B, NY, NX, NZ;  // image [B][NY][NX][NZ]
  int ny, nx, nz;     // current sub-array at the corner of every item
};

struct DtJobs8 {
  const float2* src[8];
  float2* dst[8];
  DtFilt f[8];
  float scale;
};

// Orthogonal combination of the eight tree values (tree index 4 tz + 2 tx +
// ty, a = 0, b = 1) of one detail coefficient into the real and imaginary
// parts of four complex coefficients (rows u0, v0, ..., u3, v3): the 3-D
// complex wavelet is the product over the axes of (tree a + j tree b), with
// the x and y factors optionally conjugated (signs sx, sy = ++, +-, -+, --):
// u = (aaa - sx sy abb - sx bba - sy bab)/2, v = (sx aba + sy aab + baa - sx sy bbb)/2.
__device__ __forceinline__ float dt3_c(int row, int t) {
  const int k = row >> 1;
  const float sx = (k & 2) ? -1.f : 1.f, sy = (k & 1) ? -1.f : 1.f;
  if ((row & 1) == 0) {
    switch (t) {
      case 0: return 0.5f;
      case 3: return -0.5f * sx * sy;
      case 6: return -0.5f * sx;
      case 5: return -0.5f * sy;
      default: return 0.f;
    }
  }
  switch (t) {
    case 2: return 0.5f * sx;
    case 1: return 0.5f * sy;
    case 4: return 0.5f;
    case 7: return -0.5f * sx * sy;
    default: return 0.f;
  }
}

template <bool SHRINK>
__device__ __forceinline__ void dt3_group(float2 (&w)[8], float tau2, double& acc) {
  float2 c[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    c[r] = make_float2(0.f, 0.f);
#pragma unroll
    for (int t = 0; t < 8; ++t) fma2(c[r], dt3_c(r, t), w[t]);
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const float2 u = c[2 * k], v = c[2 * k + 1];
    const float m = sqrtf(u.x * u.x + u.y * u.y + v.x * v.x + v.y * v.y);
    if (!SHRINK) {
      acc += 0.35355339059327376220 * (double)m;   // 2^(-3/2): the trees' Parseval scale
    } else {
      const float sc = m > tau2 ? 1.f - tau2 / m : 0.f;
      c[2 * k] = cscale(u, sc);
      c[2 * k + 1] = cscale(v, sc);
    }
  }
  if (SHRINK) {
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      w[t] = make_float2(0.f, 0.f);
#pragma unroll
      for (int r = 0; r < 8; ++r) fma2(w[t], dt3_c(r, t), c[r]);
    }
  }
}

__device__ __forceinline__ int64_t dt3_off(const Dt3Geom& g, int b, int y, int x, int n) {
  return (((int64_t)b * g.NY + y) * g.NX + x) * g.NZ + n;
}

// Analysis along one axis (0 depth, 1 x, 2 y) of the corner sub-array; the
// depth index runs fastest for the lateral axes (coalesced).
template <int AXIS>
__global__ void afb3_kernel(Dt3Geom g, DtJobs8 J) {
  const int j = blockIdx.y;
  const int len = AXIS == 0 ? g.nz : AXIS == 1 ? g.nx : g.ny;
  const int h = len / 2;
  const int64_t stride = AXIS == 0 ? 1 : AXIS == 1 ? (int64_t)g.NZ : (int64_t)g.NX * g.NZ;
  const int a0 = AXIS == 0 ? h : g.nz;                 // fastest index range
  const int a1 = AXIS == 1 ? h : g.nx;
  const int a2 = AXIS == 2 ? h : g.ny;
  const int64_t total = (int64_t)g.B * a2 * a1 * a0;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int i0 = (int)(t % a0);
    int64_t r = t / a0;
    const int i1 = (int)(r % a1);
    r /= a1;
    const int i2 = (int)(r % a2);
    const int b = (int)(r / a2);
    const int n = AXIS == 0 ? 0 : i0, x = AXIS == 1 ? 0 : i1, y = AXIS == 2 ? 0 : i2;
    const int i = AXIS == 0 ? i0 : AXIS == 1 ? i1 : i2;
    const int64_t base = dt3_off(g, b, y, x, n);
    float2 lo, hi;
    afb_line(J.f[j], J.src[j] + base, stride, len, i, lo, hi);
    J.dst[j][base + (int64_t)i * stride] = lo;
    J.dst[j][base + (int64_t)(h + i) * stride] = hi;
  }
}

// Synthesis along one axis; ACC sums job pairs (2y, 2y + 1) into dst[2y].
template <int AXIS, bool ACC>
__global__ void sfb3_kernel(Dt3Geom g, DtJobs8 J) {
  const int j = blockIdx.y * (ACC ? 2 : 1);
  const int len = AXIS == 0 ? g.nz : AXIS == 1 ? g.nx : g.ny;
  const int64_t stride = AXIS == 0 ? 1 : AXIS == 1 ? (int64_t)g.NZ : (int64_t)g.NX * g.NZ;
  const int64_t total = (int64_t)g.B * g.ny * g.nx * g.nz;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int n = (int)(t % g.nz);
    int64_t r = t / g.nz;
    const int x = (int)(r % g.nx);
    r /= g.nx;
    const int y = (int)(r % g.ny);
    const int b = (int)(r / g.ny);
    const int m = AXIS == 0 ? n : AXIS == 1 ? x : y;
    const int64_t base = dt3_off(g, b, AXIS == 2 ? 0 : y, AXIS == 1 ? 0 : x, AXIS == 0 ? 0 : n);
    float2 v = sfb_line(J.f[j], J.src[j] + base, stride, len, m);
    if (ACC) {
      const float2 w = sfb_line(J.f[j + 1], J.src[j + 1] + base, stride, len, m);
      v = make_float2(v.x + w.x, v.y + w.y);
    }
    J.dst[j][base + (int64_t)m * stride] = make_float2(J.scale * v.x, J.scale * v.y);
  }
}

// Lateral synthesis of the volume along x (AXIS 1) or y (AXIS 2) with a
// sliding register window.  Per output, sfb3_kernel fetches one input row per
// tap; rows 16 KB (x) or n_x n_z samples (y) apart are not held by the caches
// between neighbouring outputs, so each input came from memory about once per
// tap.  Outputs 2p and 2p + 1 read the same NT/2 rows i = p - NT/2 + 1 .. p of
// each band, so a thread that walks RP output pairs along the axis (one depth
// lane, one position of the other lateral axis) loads every row once, plus
// NT/2 - 1 rows at the start of its run, with no LDS and no barrier.  Window
// slots are fixed at compile time (the walk is unrolled).  Taps are applied
// in sfb_line's order and the per-tree sums added as in sfb3_kernel: the same
// result bit for bit.
template <int AXIS, bool ACC, int NT>
__global__ void __launch_bounds__(256) sfb3_window(Dt3Geom g, DtJobs8 J) {
  static_assert(AXIS == 1 || AXIS == 2, "lateral axes only");
  constexpr int W = NT / 2, RP = 16;
  constexpr int NS = ACC ? 2 : 1;
  const int j = blockIdx.y * NS;
  const int len = AXIS == 1 ? g.nx : g.ny, h = len / 2;
  const int others = AXIS == 1 ? g.ny : g.nx;
  const int runs = (h + RP - 1) / RP;
  const int64_t stride = AXIS == 1 ? (int64_t)g.NZ : (int64_t)g.NX * g.NZ;
  const int64_t total = (int64_t)g.B * others * runs * g.nz;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int n = (int)(t % g.nz);
    int64_t r = t / g.nz;
    const int run = (int)(r % runs);
    r /= runs;
    const int other = (int)(r % others);
    const int b = (int)(r / others);
    const int64_t item = (AXIS == 1 ? (((int64_t)b * g.NY + other) * g.NX) * g.NZ
                                    : ((int64_t)b * g.NY * g.NX + other) * g.NZ) + n;
    const int p0 = run * RP;
    // slot u % W holds band row p0 - W + 1 + u (mod h)
    float2 lo[NS][W], hi[NS][W];
#pragma unroll
    for (int u = 0; u < W - 1; ++u) {
      int i = (p0 - W + 1 + u) % h;
      if (i < 0) i += h;
#pragma unroll
      for (int q = 0; q < NS; ++q) {
        lo[q][u % W] = J.src[j + q][item + (int64_t)i * stride];
        hi[q][u % W] = J.src[j + q][item + (int64_t)(h + i) * stride];
      }
    }
#pragma unroll
    for (int sp = 0; sp < RP; ++sp) {
      const int p = p0 + sp;
      if (p < h) {
#pragma unroll
        for (int q = 0; q < NS; ++q) {
          lo[q][(W - 1 + sp) % W] = J.src[j + q][item + (int64_t)p * stride];
          hi[q][(W - 1 + sp) % W] = J.src[j + q][item + (int64_t)(h + p) * stride];
        }
#pragma unroll
        for (int odd = 0; odd < 2; ++odd) {
          float2 v = make_float2(0.f, 0.f);
#pragma unroll
          for (int q = 0; q < NS; ++q) {
            const DtFilt& f = J.f[j + q];
            float2 x = make_float2(0.f, 0.f);
#pragma unroll
            for (int k = odd; k < NT; k += 2) {
              const int slot = (W - 1 + sp - (k >> 1)) % W;
              fma2(x, f.h0[k], lo[q][slot]);
              fma2(x, f.h1[k], hi[q][slot]);
            }
            v = q == 0 ? x : make_float2(v.x + x.x, v.y + x.y);
          }
          J.dst[j][item + (int64_t)(2 * p + odd) * stride] = make_float2(J.scale * v.x, J.scale * v.y);
        }
      }
    }
  }
}

// y analysis of all eight trees in one thread with the level's detail bands
// combined and shrunk (or summed) on the spot, as afb_lateral4_kernel.
template <bool SHRINK>
__global__ void afb3_y8_kernel(Dt3Geom g, DtJobs8 J, float tau2, double* partial) {
  __shared__ double sh[16];
  const int h = g.ny / 2, hx = g.nx / 2, hz = g.nz / 2;
  const int64_t total = (int64_t)g.B * h * g.nx * g.nz;
  const int64_t stride = (int64_t)g.NX * g.NZ;
  double acc = 0.0;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int n = (int)(t % g.nz);
    int64_t r = t / g.nz;
    const int x = (int)(r % g.nx);
    r /= g.nx;
    const int i = (int)(r % h);
    const int b = (int)(r / h);
    const int64_t base = dt3_off(g, b, 0, x, n);
    float2 lo[8], hi[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) afb_line(J.f[k], J.src[k] + base, stride, g.ny, i, lo[k], hi[k]);
    const bool low3 = n < hz && x < hx;   // y-low output of the all-low band continues to the next level
    if (!low3) dt3_group<SHRINK>(lo, tau2, acc);
    dt3_group<SHRINK>(hi, tau2, acc);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (SHRINK || low3) J.dst[k][base + (int64_t)i * stride] = lo[k];
      if (SHRINK) J.dst[k][base + (int64_t)(h + i) * stride] = hi[k];
    }
  }
  if (!SHRINK) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += sh[k];
      partial[blockIdx.x] = s;
    }
  }
}

// The first level's y analysis with a sliding register window: there the
// eight trees read four sources (trees 2q and 2q + 1 filter the same staging
// buffer with the two filters), and output i reads rows 2i .. 2i + NT - 1,
// so a thread walking RP outputs along y (one depth lane, one x) keeps NT
// rows of each source in registers and loads two new rows per output.  Taps
// in afb_line's order: the coefficients, and every value written, are those
// of afb3_y8_kernel bit for bit (the value pass's FP64 partial sums add the
// same terms in another order).
template <bool SHRINK, int NT>
__global__ void __launch_bounds__(256) afb3_y8_window(Dt3Geom g, DtJobs8 J, float tau2, double* partial) {
  constexpr int RP = 16;
  __shared__ double sh[16];
  const int len = g.ny, h = g.ny / 2, hx = g.nx / 2, hz = g.nz / 2;
  const int runs = (h + RP - 1) / RP;
  const int64_t total = (int64_t)g.B * runs * g.nx * g.nz;
  const int64_t stride = (int64_t)g.NX * g.NZ;
  double acc = 0.0;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int n = (int)(t % g.nz);
    int64_t r = t / g.nz;
    const int x = (int)(r % g.nx);
    r /= g.nx;
    const int run = (int)(r % runs);
    const int b = (int)(r / runs);
    const int64_t base = dt3_off(g, b, 0, x, n);
    const int i0 = run * RP;
    const bool low3 = n < hz && x < hx;   // y-low output of the all-low band continues to the next level
    // slot u % NT holds row (2 i0 + u) mod len of source q (trees 2q, 2q + 1)
    float2 win[4][NT];
#pragma unroll
    for (int u = 0; u < NT - 2; ++u) {
      const int row = (2 * i0 + u) % len;
#pragma unroll
      for (int q = 0; q < 4; ++q) win[q][u % NT] = J.src[2 * q][base + (int64_t)row * stride];
    }
#pragma unroll
    for (int si = 0; si < RP; ++si) {
      const int i = i0 + si;
      if (i < h) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int u = 2 * si + NT - 2 + e;
          const int row = (2 * i0 + u) % len;
#pragma unroll
          for (int q = 0; q < 4; ++q) win[q][u % NT] = J.src[2 * q][base + (int64_t)row * stride];
        }
        float2 lo[8], hi[8];
#pragma unroll
        for (int k8 = 0; k8 < 8; ++k8) {
          const DtFilt& f = J.f[k8];
          lo[k8] = make_float2(0.f, 0.f);
          hi[k8] = make_float2(0.f, 0.f);
#pragma unroll
          for (int k = 0; k < NT; ++k) {
            const float2 v = win[k8 >> 1][(2 * si + k) % NT];
            fma2(lo[k8], f.h0[k], v);
            fma2(hi[k8], f.h1[k], v);
          }
        }
        if (!low3) dt3_group<SHRINK>(lo, tau2, acc);
        dt3_group<SHRINK>(hi, tau2, acc);
#pragma unroll
        for (int k8 = 0; k8 < 8; ++k8) {
          if (SHRINK || low3) J.dst[k8][base + (int64_t)i * stride] = lo[k8];
          if (SHRINK) J.dst[k8][base + (int64_t)(h + i) * stride] = hi[k8];
        }
      }
    }
  }
  if (!SHRINK) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) sh[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      for (int k = 0; k < (int)(blockDim.x >> 6); ++k) s += sh[k];
      partial[blockIdx.x] = s;
    }
  }
}

// x analysis with a sliding register window (one job per blockIdx.y, one
// source and one filter each): output i reads rows 2i .. 2i + NT - 1.
template <int NT>
__global__ void __launch_bounds__(256) afb3_x_window(Dt3Geom g, DtJobs8 J) {
  constexpr int RP = 16;
  const int j = blockIdx.y;
  const DtFilt& f = J.f[j];
  const int len = g.nx, h = g.nx / 2;
  const int runs = (h + RP - 1) / RP;
  const int64_t total = (int64_t)g.B * g.ny * runs * g.nz;
  const int64_t stride = g.NZ;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
    const int n = (int)(t % g.nz);
    int64_t r = t / g.nz;
    const int run = (int)(r % runs);
    r /= runs;
    const int y = (int)(r % g.ny);
    const int b = (int)(r / g.ny);
    const int64_t base = dt3_off(g, b, y, 0, n);
    const int i0 = run * RP;
    float2 win[NT];
#pragma unroll
    for (int u = 0; u < NT - 2; ++u) win[u % NT] = J.src[j][base + (int64_t)((2 * i0 + u) % len) * stride];
#pragma unroll
    for (int si = 0; si < RP; ++si) {
      const int i = i0 + si;
      if (i < h) {
#pragma unroll
        for (int e = 0; e < 2; ++e) {
          const int u = 2 * si + NT - 2 + e;
          win[u % NT] = J.src[j][base + (int64_t)((2 * i0 + u) % len) * stride];
        }
        float2 lo = make_float2(0.f, 0.f), hi = make_float2(0.f, 0.f);
#pragma unroll
        for (int k = 0; k < NT; ++k) {
          const float2 v = win[(2 * si + k) % NT];
          fma2(lo, f.h0[k], v);
          fma2(hi, f.h1[k], v);
        }
        J.dst[j][base + (int64_t)i * stride] = lo;
        J.dst[j][base + (int64_t)(h + i) * stride] = hi;
      }
    }
  }
}

// Workspace of the volume transform: 8 trees, then staging buffers S (8) and
// U (8), one image each.
struct Dt3Work {
  float2* tree[8];
  float2* S[8];
  float2* U[8];
};

Dt3Work dt3_work(float2* work, int64_t n) {
  Dt3Work w;
  for (int t = 0; t < 8; ++t) {
    w.tree[t] = work + t * n;
    w.S[t] = work + (8 + t) * n;
    w.U[t] = work + (16 + t) * n;
  }
  return w;
}

// Analysis of the eight trees; mode 0 shrinks the details by tau2, mode 1
// writes the block partials of sum |W x| (value pass).
hipError_t dt3_analysis(const Dt3Geom& g0, int levels, const float2* v, const Dt3Work& w, int mode, float tau2,
                        double* partial, hipStream_t s) {
  const DtFilters& F = filters();
  Dt3Geom g = g0;
  for (int lev = 0; lev < levels; ++lev) {
    const DtFilt* fs = lev == 0 ? F.first : F.later;
    DtJobs8 jz{}, jx{}, jy{};
    int nz_jobs, nx_jobs;
    if (lev == 0) {
      // depth filters once per depth tree, x filters once per (depth, x) pair
      nz_jobs = 2;
      for (int p = 0; p < 2; ++p) {
        jz.src[p] = v;
        jz.dst[p] = w.S[p];
        jz.f[p] = fs[p];
      }
      nx_jobs = 4;
      for (int p = 0; p < 4; ++p) {
        jx.src[p] = w.S[p >> 1];
        jx.dst[p] = w.U[p];
        jx.f[p] = fs[p & 1];
      }
      for (int t = 0; t < 8; ++t) {
        jy.src[t] = w.U[t >> 1];
        jy.dst[t] = w.tree[t];
        jy.f[t] = fs[t & 1];
      }
    } else {
      nz_jobs = nx_jobs = 8;
      for (int t = 0; t < 8; ++t) {
        jz.src[t] = w.tree[t];
        jz.dst[t] = w.S[t];
        jz.f[t] = fs[t >> 2];
        jx.src[t] = w.S[t];
        jx.dst[t] = w.U[t];
        jx.f[t] = fs[(t >> 1) & 1];
        jy.src[t] = w.U[t];
        jy.dst[t] = w.tree[t];
        jy.f[t] = fs[t & 1];
      }
    }
    const int64_t nzw = (int64_t)g.B * g.ny * g.nx * (g.nz / 2), nxw = (int64_t)g.B * g.ny * (g.nx / 2) * g.nz;
    const int64_t nyw = (int64_t)g.B * (g.ny / 2) * g.nx * g.nz;
    hipLaunchKernelGGL(afb3_kernel<0>, dim3(dt_grid_y(nzw, nz_jobs), nz_jobs), dim3(256), 0, s, g, jz);
    // x: register-window kernel for the 8- and 12-tap filters
    const int ntx = jx.f[0].n;
    const int64_t tw = (int64_t)g.B * g.ny * ((g.nx / 2 + 15) / 16) * g.nz;
    bool xw = (ntx == 8 || ntx == 12) && tw >= DT_WINDOW_MIN_THREADS;
    for (int q = 0; q < nx_jobs; ++q) xw = xw && jx.f[q].n == ntx;
    if (xw) {
      if (ntx == 8)
        hipLaunchKernelGGL(afb3_x_window<8>, dim3(dt_grid_y(tw, nx_jobs), nx_jobs), dim3(256), 0, s, g, jx);
      else
        hipLaunchKernelGGL(afb3_x_window<12>, dim3(dt_grid_y(tw, nx_jobs), nx_jobs), dim3(256), 0, s, g, jx);
    } else {
      hipLaunchKernelGGL(afb3_kernel<1>, dim3(dt_grid_y(nxw, nx_jobs), nx_jobs), dim3(256), 0, s, g, jx);
    }
    // y: at the first level the trees read four sources with two 8-tap filters: register window
    const bool yw = lev == 0 && fs[0].n == 8 && fs[1].n == 8 &&
                    (int64_t)g.B * ((g.ny / 2 + 15) / 16) * g.nx * g.nz >= DT_WINDOW_MIN_THREADS;
    if (mode == 0) {
      if (yw)
        hipLaunchKernelGGL((afb3_y8_window<true, 8>), dim3(dt_grid(nyw)), dim3(256), 0, s, g, jy, tau2, nullptr);
      else
        hipLaunchKernelGGL((afb3_y8_kernel<true>), dim3(dt_grid(nyw)), dim3(256), 0, s, g, jy, tau2, nullptr);
    } else {
      if (yw)
        hipLaunchKernelGGL((afb3_y8_window<false, 8>), dim3(dt_grid(nyw)), dim3(256), 0, s, g, jy, 0.f, partial);
      else
        hipLaunchKernelGGL((afb3_y8_kernel<false>), dim3(dt_grid(nyw)), dim3(256), 0, s, g, jy, 0.f, partial);
      partial += dt_grid(nyw);
    }
    g.ny /= 2;
    g.nx /= 2;
    g.nz /= 2;
  }
  return hipGetLastError();
}

}  // namespace

int dtcwt_partials(const ProxGeom& pg, int levels) {
  int n = 0;
  if (pg.lateral_dims == 2) {
    int64_t ny = pg.Ny, nx = pg.Nx, nz = pg.Nz;
    for (int lev = 0; lev < levels; ++lev) {
      n += dt_grid((int64_t)pg.B * (ny / 2) * nx * nz);
      ny /= 2;
      nx /= 2;
      nz /= 2;
    }
    return n;
  }
  DtGeom g{pg.B, pg.Nx, pg.Nz, pg.Nx, pg.Nz};
  for (int lev = 0; lev < levels; ++lev) {
    n += dt_grid((int64_t)g.B * (g.nx / 2) * g.nz);
    g.nx /= 2;
    g.nz /= 2;
  }
  return n;
}

size_t dtcwt_work_elems(const ProxGeom& pg) {
  const size_t n = (size_t)pg.B * pg.Ny * pg.Nx * pg.Nz;
  return (pg.lateral_dims == 2 ? 24 : 8) * n;
}

// Lateral synthesis pass of the volume: the register-window kernel for the 8-
// and 12-tap filters on large enough sub-arrays, else the per-tap one.
template <int AXIS, bool ACC>
void sfb3_lateral(const Dt3Geom& g, const DtJobs8& J, int jobs, hipStream_t s) {
  const int nt = J.f[0].n;
  bool same = true;
  for (int q = 0; q < jobs * (ACC ? 2 : 1); ++q) same = same && J.f[q].n == nt;
  const int len = AXIS == 1 ? g.nx : g.ny, others = AXIS == 1 ? g.ny : g.nx;
  const int64_t total = (int64_t)g.B * others * ((len / 2 + 15) / 16) * g.nz;
  if (same && (nt == 8 || nt == 12) && total >= DT_WINDOW_MIN_THREADS) {
    if (nt == 8)
      hipLaunchKernelGGL((sfb3_window<AXIS, ACC, 8>), dim3(dt_grid_y(total, jobs), jobs), dim3(256), 0, s, g, J);
    else
      hipLaunchKernelGGL((sfb3_window<AXIS, ACC, 12>), dim3(dt_grid_y(total, jobs), jobs), dim3(256), 0, s, g, J);
    return;
  }
  const int64_t nn = (int64_t)g.B * g.ny * g.nx * g.nz;
  hipLaunchKernelGGL((sfb3_kernel<AXIS, ACC>), dim3(dt_grid_y(nn, jobs), jobs), dim3(256), 0, s, g, J);
}

hipError_t launch_prox_dtcwt3(const ProxGeom& pg, int levels, const float2* v, float2* z, float tau, float2* work,
                              hipStream_t s) {
  const int64_t n = (int64_t)pg.B * pg.Ny * pg.Nx * pg.Nz;
  const Dt3Work w = dt3_work(work, n);
  const Dt3Geom g0{pg.B, pg.Ny, pg.Nx, pg.Nz, pg.Ny, pg.Nx, pg.Nz};
  // unscaled trees: soft threshold 2^(3/2) tau, synthesis sum scaled by 1/8
  hipError_t e = dt3_analysis(g0, levels, v, w, 0, 2.8284271247461900976f * tau, nullptr, s);
  if (e != hipSuccess) return e;
  const DtFilters& F = filters();
  for (int lev = levels - 1; lev >= 0; --lev) {
    Dt3Geom gl = g0;
    gl.ny = pg.Ny >> lev;
    gl.nx = pg.Nx >> lev;
    gl.nz = pg.Nz >> lev;
    const DtFilt* fs = lev == 0 ? F.first : F.later;
    const int64_t nn = (int64_t)gl.B * gl.ny * gl.nx * gl.nz;
    DtJobs8 jy{}, jx{}, jz{};
    jy.scale = jx.scale = jz.scale = 1.f;
    if (lev > 0) {
      for (int t = 0; t < 8; ++t) {
        jy.src[t] = w.tree[t];
        jy.dst[t] = w.S[t];
        jy.f[t] = fs[t & 1];
        jx.src[t] = w.S[t];
        jx.dst[t] = w.U[t];
        jx.f[t] = fs[(t >> 1) & 1];
        jz.src[t] = w.U[t];
        jz.dst[t] = w.tree[t];
        jz.f[t] = fs[t >> 2];
      }
      sfb3_lateral<2, false>(gl, jy, 8, s);
      sfb3_lateral<1, false>(gl, jx, 8, s);
      hipLaunchKernelGGL((sfb3_kernel<0, false>), dim3(dt_grid_y(nn, 8), 8), dim3(256), 0, s, gl, jz);
    } else {
      // y: trees (p, ty = a) + (p, ty = b) -> S[2q], p = 4 tz + 2 tx = 2q; x: S[4 tz] + S[4 tz + 2] -> U[tz];
      // depth: U[a] + U[b], times 1/8, -> z
      for (int t = 0; t < 8; ++t) {
        jy.src[t] = w.tree[t];
        jy.dst[t] = w.S[t];
        jy.f[t] = fs[t & 1];
      }
      for (int q = 0; q < 4; ++q) {
        jx.src[q] = w.S[2 * q];
        jx.dst[q] = w.U[q];
        jx.f[q] = fs[q & 1];
      }
      jz.src[0] = w.U[0];
      jz.src[1] = w.U[2];
      jz.dst[0] = z;
      jz.f[0] = fs[0];
      jz.f[1] = fs[1];
      jz.scale = 0.125f;
      sfb3_lateral<2, true>(gl, jy, 4, s);
      sfb3_lateral<1, true>(gl, jx, 2, s);
      hipLaunchKernelGGL((sfb3_kernel<0, true>), dim3(dt_grid_y(nn, 1), 1), dim3(256), 0, s, gl, jz);
    }
  }
  return hipGetLastError();
}

hipError_t launch_prox_dtcwt(const ProxGeom& pg, int levels, const float2* v, float2* z, float tau, float2* work,
                             hipStream_t s) {
  if (pg.lateral_dims == 2) return launch_prox_dtcwt3(pg, levels, v, z, tau, work, s);
  const int64_t n = (int64_t)pg.B * pg.Nx * pg.Nz;
  const DtWork w = dt_work(work, n);
  const DtGeom g0{pg.B, pg.Nx, pg.Nz, pg.Nx, pg.Nz};
  hipError_t e = dt_analysis(g0, levels, v, w, 0, 2.f * tau, nullptr, s);
  if (e != hipSuccess) return e;
  // synthesis, coarsest level first; level 1 sums the two trees of each depth
  // filter after their lateral passes and the two depth filters at the end,
  // with the 1/4 of the Parseval normalisation
  const DtFilters& F = filters();
  for (int lev = levels - 1; lev >= 0; --lev) {
    DtGeom gl = g0;
    gl.nx = pg.Nx >> lev;
    gl.nz = pg.Nz >> lev;
    const DtFilt* fs = lev == 0 ? F.first : F.later;
    const int64_t nn = (int64_t)gl.B * gl.nx * gl.nz;
    DtJobs jl{}, jd{};
    jl.scale = jd.scale = 1.f;
    for (int t = 0; t < 4; ++t) {
      jl.src[t] = w.tr.t[t];
      jl.dst[t] = w.tmp[t];
      jl.f[t] = fs[t & 1];
    }
    if (lev > 0) {
      for (int t = 0; t < 4; ++t) {
        jd.src[t] = w.tmp[t];
        jd.dst[t] = w.tr.t[t];
        jd.f[t] = fs[t >> 1];
      }
      hipLaunchKernelGGL((sfb_lateral_tiled<false>), dt_sfb_grid(gl, 4), dim3(256), 0, s, gl, jl);
      hipLaunchKernelGGL((sfb_depth_kernel<false>), dim3(dt_grid_y(nn, 4), 4), dim3(256), 0, s, gl, jd);
    } else {
      // tmp[0] = lat(aa) + lat(ab), tmp[2] = lat(ba) + lat(bb)
      hipLaunchKernelGGL((sfb_lateral_tiled<true>), dt_sfb_grid(gl, 2), dim3(256), 0, s, gl, jl);
      jd.src[0] = w.tmp[0];
      jd.src[1] = w.tmp[2];
      jd.dst[0] = jd.dst[1] = z;
      jd.f[0] = fs[0];
      jd.f[1] = fs[1];
      jd.scale = 0.25f;
      hipLaunchKernelGGL((sfb_depth_kernel<true>), dim3(dt_grid_y(nn, 1), 1), dim3(256), 0, s, gl, jd);
    }
  }
  return hipGetLastError();
}

hipError_t launch_dtcwt_value(const ProxGeom& pg, int levels, const float2* x, float2* work, double* partial,
                              hipStream_t s) {
  if (pg.lateral_dims == 2) {
    const int64_t n = (int64_t)pg.B * pg.Ny * pg.Nx * pg.Nz;
    const Dt3Geom g0{pg.B, pg.Ny, pg.Nx, pg.Nz, pg.Ny, pg.Nx, pg.Nz};
    return dt3_analysis(g0, levels, x, dt3_work(work, n), 1, 0.f, partial, s);
  }
  const int64_t n = (int64_t)pg.B * pg.Nx * pg.Nz;
  const DtWork w = dt_work(work, n);
  const DtGeom g0{pg.B, pg.Nx, pg.Nz, pg.Nx, pg.Nz};
  return dt_analysis(g0, levels, x, w, 1, 0.f, partial, s);
}

// Host copies of the designed filters (for the library's own checks).
void dtcwt_filter_taps(int which, float* h0, int* n) {
  const DtFilters& F = filters();
  const DtFilt& f = which == 0 ? F.first[0] : which == 1 ? F.first[1] : which == 2 ? F.later[0] : F.later[1];
  *n = f.n;
  for (int k = 0; k < f.n; ++k) h0[k] = f.h0[k];
}
