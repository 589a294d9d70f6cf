// Per-lateral-frequency NUFFT of the ISAM resampling (Sec. 2.1, eq. (5)-(6)):
// for each column q the depth profile is deapodised, centred at n_c and
// zero-padded onto a sigma-times oversampled grid of K cells, transformed by
// an in-LDS FFT, and interpolated with J Kaiser-Bessel taps at the grid
// coordinate t_m(q) = K dz beta_m(q) / (2 pi), beta = sqrt(4 k_m^2 - q^2);
// the beam, focus and dispersion filter is applied on the way out.
//
// The adjoint spreads samples back onto the grid without atomics: every grid
// cell gathers, in increasing m, the samples whose J-tap window covers it.
// t_m(q) increases with m, so those samples form a contiguous run found by a
// binary search plus a moving pointer; the sum order is fixed, so the result
// is bitwise reproducible.
//
// Coordinates are formed in FP64 (t reaches ~1e4 cells and its fraction
// must be good to ~1e-7); the KB weights come from degree-9 polynomial
// pieces, one per tap, in x = 2 frac(t) - 1, evaluated in FP32.
#include "oct_fft.h"

namespace {

constexpr int KBD = OCT_KB_DEG;

__device__ __forceinline__ float kb_poly(const float* __restrict__ c, float x) {
  float w = c[KBD];
#pragma unroll
  for (int d = KBD - 1; d >= 0; --d) w = fmaf(w, x, c[d]);
  return w;
}

// Filter H(m, q) = beam(q) e^{j(-2 k_m z_f + Omega_m)} e^{j beta (z_f - n_c dz)}.
__device__ __forceinline__ float2 filter_h(const NufftArgs& a, int m, float bq, double beta) {
  float2 h = a.phase[m];
  h.x *= bq;
  h.y *= bq;
  if (a.df != 0.0) {
    double sn, cs;
    sincos(beta * a.df, &sn, &cs);
    h = cmul(h, make_float2((float)cs, (float)sn));
  }
  return h;
}

template <int J, bool R7>
__global__ void __launch_bounds__(1024) nufft_fwd_kernel(NufftArgs a, const float2* __restrict__ X1,
                                                         float2* __restrict__ W) {
  extern __shared__ float2 grid[];
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int col = blockIdx.x;
  const int lat = col % a.Nlat;
  const int K = a.K, Nz = a.Nz, nc = a.nc;
  const float2* __restrict__ src = X1 + (int64_t)col * Nz;

  // n' = n - n_c placed at n' mod K; cells [Nz - nc, K - nc) stay zero.
  for (int i = tid; i < K - Nz; i += nthr) grid[Nz - nc + i] = make_float2(0.f, 0.f);
  for (int n = tid; n < Nz; n += nthr) {
    int idx = n - nc;
    if (idx < 0) idx += K;
    grid[idx] = cscale(src[n], a.deap[n]);
  }
  __syncthreads();
  fft_rows<R7, false>(grid, 1, K, a.fK, a.twK, tid, nthr);

  const double q2 = a.q2[lat];
  const float bq = a.beam[lat];
  float2* __restrict__ out = W + (int64_t)col * a.Mk;
  for (int m = tid; m < a.Mk; m += nthr) {
    const double arg = a.k2x4[m] - q2;
    float2 res = make_float2(0.f, 0.f);
    if (arg > 0.0) {
      const double beta = sqrt(arg);
      const double t = a.ct * beta;
      const double fl = floor(t);
      const float x = (float)(2.0 * (t - fl) - 1.0);
      int c0 = ((int)fl - J / 2 + 1) % K;
      if (c0 < 0) c0 += K;
      float2 acc = make_float2(0.f, 0.f);
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const float w = kb_poly(a.kbc + j * (KBD + 1), x);
        int idx = c0 + j;
        if (idx >= K) idx -= K;
        const float2 gv = grid[idx];
        acc.x = fmaf(w, gv.x, acc.x);
        acc.y = fmaf(w, gv.y, acc.y);
      }
      res = cmul(filter_h(a, m, bq, beta), acc);
    }
    out[m] = res;
  }
}

constexpr int EVANESCENT = -(1 << 29);

template <int J, bool R7>
__global__ void __launch_bounds__(1024) nufft_adj_kernel(NufftArgs a, const float2* __restrict__ Rh,
                                                         float2* __restrict__ X) {
  extern __shared__ float4 smem4[];
  __shared__ float kc[J * (KBD + 1)];
  float2* grid = reinterpret_cast<float2*>(smem4);
  float2* us = grid + a.K;
  int* bm = reinterpret_cast<int*>(us + a.Mk);
  float* xm = reinterpret_cast<float*>(bm + a.Mk);
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int col = blockIdx.x;
  const int lat = col % a.Nlat;
  const int K = a.K, Mk = a.Mk, Nz = a.Nz, nc = a.nc;

  for (int i = tid; i < J * (KBD + 1); i += nthr) kc[i] = a.kbc[i];
  const double q2 = a.q2[lat];
  const float bq = a.beam[lat];
  const float2* __restrict__ rin = Rh + (int64_t)col * Mk;
  for (int m = tid; m < Mk; m += nthr) {
    const double arg = a.k2x4[m] - q2;
    if (arg > 0.0) {
      const double beta = sqrt(arg);
      const double t = a.ct * beta;
      const double fl = floor(t);
      bm[m] = (int)fl;
      xm[m] = (float)(2.0 * (t - fl) - 1.0);
      us[m] = cmul(cconj(filter_h(a, m, bq, beta)), rin[m]);
    } else {
      bm[m] = EVANESCENT;
      xm[m] = 0.f;
      us[m] = make_float2(0.f, 0.f);
    }
  }
  __syncthreads();

  // first propagating sample (evanescent ones form a prefix: lowest k)
  int lo = 0, hi = Mk;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (bm[mid] == EVANESCENT) lo = mid + 1; else hi = mid;
  }
  const int mf = lo;
  int umin = 0, umax = -1;
  if (mf < Mk) {
    umin = bm[mf] - J / 2 + 1;
    umax = bm[Mk - 1] + J / 2;
  }
  const int span = umax - umin + 1;
  const int nph = span > K ? (span + K - 1) / K : 1;
  const double q2c = q2;
  for (int ph = 0; ph < nph; ++ph) {
    const int pbeg = umin + ph * K;
    int pend = pbeg + K;
    if (ph > 0) pend = min(pend, umax + 1);
    // consecutive lanes take consecutive cells, so their samples are
    // consecutive too (conflict-free LDS reads)
    for (int u = pbeg + tid; u < pend; u += nthr) {
      const int key = u - J / 2;   // first contributor: smallest m with bm[m] >= key
      int p = mf;
      if (mf < Mk) {
        // invert t = ct sqrt(4 k^2 - q^2) for the starting sample, then walk
        // to the exact boundary on the stored base cells
        const double bta = fmax((double)key, 0.0) / a.ct;
        const double km = 0.5 * sqrt(bta * bta + q2c);
        double mstar = floor((km - a.k_min) / a.dk);
        mstar = fmin(fmax(mstar, (double)mf), (double)Mk);
        p = (int)mstar;
        while (p > mf && bm[p - 1] >= key) --p;
        while (p < Mk && bm[p] < key) ++p;
      }
      float2 acc = make_float2(0.f, 0.f);
      for (int m = p; m < Mk && bm[m] <= u + J / 2 - 1; ++m) {
        const int j = u - (bm[m] - J / 2 + 1);
        const float w = kb_poly(kc + j * (KBD + 1), xm[m]);
        const float2 uv = us[m];
        acc.x = fmaf(w, uv.x, acc.x);
        acc.y = fmaf(w, uv.y, acc.y);
      }
      int g = u % K;
      if (g < 0) g += K;
      if (ph == 0) grid[g] = acc;
      else grid[g] = cadd(grid[g], acc);
    }
    __syncthreads();
  }

  fft_rows<R7, true>(grid, 1, K, a.fK, a.twK, tid, nthr);
  float2* __restrict__ dst = X + (int64_t)col * Nz;
  for (int n = tid; n < Nz; n += nthr) {
    int idx = n - nc;
    if (idx < 0) idx += K;
    dst[n] = cscale(grid[idx], a.deap[n]);
  }
}

int nufft_threads(const NufftArgs& a) {
  const int bf = a.K / a.fK.min_radix;
  const int mb = fft_maxb(a.fK);
  int nt = 256;
  while (nt < 1024 && bf > mb * nt) nt <<= 1;
  return nt;
}

}  // namespace

size_t nufft_adj_lds_bytes(const NufftArgs& a) {
  return (size_t)a.K * sizeof(float2) + (size_t)a.Mk * (sizeof(float2) + sizeof(int) + sizeof(float));
}

template <int J, bool R7>
hipError_t nufft_fwd_t(const NufftArgs& a, const float2* X1, float2* W, hipStream_t s) {
  const size_t lds = (size_t)a.K * sizeof(float2);
  hipLaunchKernelGGL((nufft_fwd_kernel<J, R7>), dim3(a.n_cols), dim3(nufft_threads(a)), lds, s, a, X1, W);
  return hipGetLastError();
}

hipError_t launch_nufft_fwd(const NufftArgs& a, const float2* X1, float2* W, hipStream_t s) {
  const bool r7 = fft_has7(a.fK);
  switch (a.J) {
    case 4: return r7 ? nufft_fwd_t<4, true>(a, X1, W, s) : nufft_fwd_t<4, false>(a, X1, W, s);
    case 6: return r7 ? nufft_fwd_t<6, true>(a, X1, W, s) : nufft_fwd_t<6, false>(a, X1, W, s);
    default: return r7 ? nufft_fwd_t<8, true>(a, X1, W, s) : nufft_fwd_t<8, false>(a, X1, W, s);
  }
}

template <int J, bool R7>
hipError_t nufft_adj_t(const NufftArgs& a, const float2* Rh, float2* X, hipStream_t s) {
  const size_t lds = nufft_adj_lds_bytes(a);
  if (lds > 64 * 1024 - 1024) {
    static bool done = false;
    if (!done) {
      hipFuncSetAttribute(reinterpret_cast<const void*>(&nufft_adj_kernel<J, R7>),
                          hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 2048);
      done = true;
    }
  }
  hipLaunchKernelGGL((nufft_adj_kernel<J, R7>), dim3(a.n_cols), dim3(nufft_threads(a)), lds, s, a, Rh, X);
  return hipGetLastError();
}

hipError_t launch_nufft_adj(const NufftArgs& a, const float2* Rh, float2* X, hipStream_t s) {
  const bool r7 = fft_has7(a.fK);
  switch (a.J) {
    case 4: return r7 ? nufft_adj_t<4, true>(a, Rh, X, s) : nufft_adj_t<4, false>(a, Rh, X, s);
    case 6: return r7 ? nufft_adj_t<6, true>(a, Rh, X, s) : nufft_adj_t<6, false>(a, Rh, X, s);
    default: return r7 ? nufft_adj_t<8, true>(a, Rh, X, s) : nufft_adj_t<8, false>(a, Rh, X, s);
  }
}
