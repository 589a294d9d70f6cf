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
// must be good to ~1e-7); the KB weights come from degree-7 polynomial
// pieces, one per tap, in x = 2 frac(t) - 1, evaluated in FP32.  The forward
// kernel keeps KPAD wrapped copies of the grid on each side of it in LDS, so
// that a sample's J taps are J consecutive cells with no per-tap wrap.
#include "oct_fft.h"

namespace {

constexpr int KBD = OCT_KB_DEG;
constexpr int KPAD = 8;   // wrapped cells on each side of the forward grid (>= J/2 + 1)

// beta = sqrt(arg), arg > 0: the FP32 reciprocal square root refined by one
// Newton step in FP64 (relative error ~2e-14, i.e. ~3e-10 cells at t ~ 1e4).
__device__ __forceinline__ double beta_of(double arg) {
  const double r0 = (double)__builtin_amdgcn_rsqf(fmaxf((float)arg, 1e-30f));
  const double h = arg * r0;            // sqrt(arg) to FP32 accuracy
  const double e = fma(-h, r0, 1.0);    // 1 - arg r0^2
  return fma(0.5 * h, e, h);
}

// Tap jj < J/2 is P(x) = E(x^2) + x O(x^2); the mirrored tap J-1-jj is
// P(-x) = E(x^2) - x O(x^2) (the window is even).  c holds E then O, each
// KBH coefficients in increasing powers of x^2.
constexpr int KBH = (KBD + 1) / 2;

__device__ __forceinline__ void kb_pair(const float* __restrict__ c, float x, float x2, float& wlo, float& whi) {
  float e = c[KBH - 1], o = c[2 * KBH - 1];
#pragma unroll
  for (int d = KBH - 2; d >= 0; --d) {
    e = fmaf(e, x2, c[d]);
    o = fmaf(o, x2, c[KBH + d]);
  }
  const float xo = x * o;
  wlo = e + xo;
  whi = e - xo;
}

// weight of tap j (0..J-1) for fraction coordinate x
template <int J>
__device__ __forceinline__ float kb_tap(const float* __restrict__ kc, int j, float x) {
  const bool lo = j < J / 2;
  const int jj = lo ? j : J - 1 - j;
  const float xs = lo ? x : -x;
  const float* c = kc + jj * 2 * KBH;
  const float x2 = xs * xs;
  float e = c[KBH - 1], o = c[2 * KBH - 1];
#pragma unroll
  for (int d = KBH - 2; d >= 0; --d) {
    e = fmaf(e, x2, c[d]);
    o = fmaf(o, x2, c[KBH + d]);
  }
  return fmaf(xs, o, e);
}

// weight of a compile-time tap j for fraction coordinate x; the coefficients
// are uniform (read once into scalar registers)
template <int J, int j>
__device__ __forceinline__ float kb_tap_ct(const float* __restrict__ kbc, float x) {
  constexpr bool lo = j < J / 2;
  constexpr int jj = lo ? j : J - 1 - j;
  const float xs = lo ? x : -x;
  const float* c = kbc + jj * 2 * KBH;
  const float x2 = xs * xs;
  float e = c[KBH - 1], o = c[2 * KBH - 1];
#pragma unroll
  for (int d = KBH - 2; d >= 0; --d) {
    e = fmaf(e, x2, c[d]);
    o = fmaf(o, x2, c[KBH + d]);
  }
  return fmaf(xs, o, e);
}

// Cell u's sum over its samples, tap-major: the samples whose tap j covers u
// are those with floor(t) = u + J/2 - 1 - j, a run [F_i, F_{i+1}) of the
// first-contributor table (i = J - 1 - j, F_i = first[u - umin + i]); the
// taps go from j = J - 1 down to 0, i.e. the samples in increasing m.
template <int J, int I>
__device__ __forceinline__ void adj_cell_taps(const float* __restrict__ kbc, const short* F, const float* xm,
                                              const float2* us, float2& s) {
  if constexpr (I < J) {
    constexpr int j = J - 1 - I;
    for (int m = F[I]; m < F[I + 1]; ++m) {   // one sample, rarely two
      const float w = kb_tap_ct<J, j>(kbc, xm[m]);
      const float2 uv = us[m];
      s.x = fmaf(w, uv.x, s.x);
      s.y = fmaf(w, uv.y, s.y);
    }
    adj_cell_taps<J, I + 1>(kbc, F, xm, us, s);
  }
}

// adj_cell_taps for two columns that share their samples' coordinates: each
// weight is evaluated once and applied to both.
template <int J, int I>
__device__ __forceinline__ void adj_cell_taps2(const float* __restrict__ kbc, const short* F, const float* xm,
                                               const float2* us0, const float2* us1, float2& s0, float2& s1) {
  if constexpr (I < J) {
    constexpr int j = J - 1 - I;
    for (int m = F[I]; m < F[I + 1]; ++m) {
      const float w = kb_tap_ct<J, j>(kbc, xm[m]);
      const float2 u0 = us0[m], u1 = us1[m];
      s0.x = fmaf(w, u0.x, s0.x);
      s0.y = fmaf(w, u0.y, s0.y);
      s1.x = fmaf(w, u1.x, s1.x);
      s1.y = fmaf(w, u1.y, s1.y);
    }
    adj_cell_taps2<J, I + 1>(kbc, F, xm, us0, us1, s0, s1);
  }
}

// Filter H(m, q) = beam(q) e^{j(-2 k_m z_f + Omega_m)} e^{j beta (z_f - n_c dz)}.
// ph = a.phase[m] (read by the caller, batched with the sample's other loads).
// The defocus phase beta (z_f - n_c dz) is reduced modulo 2 pi in FP64 (to
// ~1e-11 rad for phases up to 1e5 rad; the depth range bounds them near 4e4)
// and then taken with the FP32 sine and cosine: ~3e-7 in H, and far fewer
// registers than the FP64 sincos, whose large-argument path would otherwise
// set the kernels' register count.
__device__ __forceinline__ float2 filter_h(const NufftArgs& a, float2 ph, float bq, double beta) {
  float2 h = ph;
  h.x *= bq;
  h.y *= bq;
  if (a.df != 0.0) {
    constexpr double two_pi = 6.283185307179586, inv_two_pi = 0.15915494309189535;
    const double phase = beta * a.df;
    const float r = (float)fma(-rint(phase * inv_two_pi), two_pi, phase);
    float sn, cs;
    sincosf(r, &sn, &cs);
    h = cmul(h, make_float2(cs, sn));
  }
  return h;
}

// ---------------------------------------------------------------------------
// Half-band edge stages (oversampling 2: K = 2 Nz, n_c = Nz / 2).  The
// centred, zero-padded depth column occupies grid cells [0, K/4) (depth
// n = n_c .. Nz-1) and [3K/4, K) (n = 0 .. n_c-1).  The first Stockham stage
// of a K-point transform with radix 8 reads butterfly j's inputs from cells
// j + r K/8: only r = 0, 1, 6, 7 are nonzero, at depths j + K/4, j + 3K/8, j
// and j + K/8.  The forward grid transform therefore takes its first stage
// straight from global memory, deapodised, with no zero fill and no LDS
// round trip; symmetrically the adjoint's last stage (radix R = 8 or 4,
// outputs k + r K/R) keeps only the outputs r < R/4 and r >= 3R/4, the cells
// that hold depths, and stores them deapodised to global memory.
// ---------------------------------------------------------------------------
template <int N>
struct HalfBand {
  static constexpr CtPlan P = ct_plan(N);
  static constexpr int RL = P.r[P.ns - 1];
  static constexpr bool ok = P.ns >= 3 && P.r[0] == 8 && (RL == 8 || RL == 4) && N / RL != 8;
};

// nonzero first-stage inputs a_0, a_1, a_6, a_7 of a radix-8 butterfly
// (a_2..a_5 = 0): b_k = a_k + a_{k+4} and c_k = a_k - a_{k+4} need no adds
template <bool INV>
__device__ __forceinline__ void dft8_edges(float2 a0, float2 a1, float2 a6, float2 a7, float2* out) {
  float2 b[4] = {a0, a1, a6, a7};
  float2 c[4] = {a0, a1, make_float2(-a6.x, -a6.y), make_float2(-a7.x, -a7.y)};
  Dft<8, INV>::finish(b, c, out);
}

// Forward K-point transforms of nrows (1 or 2) deapodised, centred depth
// columns src0 (row 0) and src1 (row 1) into LDS rows buf + row rowstride.
template <int N, int MAXB>
__device__ __forceinline__ void fwd_grid_fft_half(float2* buf, int nrows, int rowstride,
                                                  const float2* __restrict__ src0, const float2* __restrict__ src1,
                                                  const float* __restrict__ deap, const FftDesc& d,
                                                  const float2* __restrict__ tw, int tid, int nthr) {
  constexpr int nb = N / 8;
  const int total = nrows * nb;
  for (int i0 = tid; i0 < total; i0 += MAXB * nthr) {
    float2 x[MAXB][4];
    float dd[MAXB][4];
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
      const int item = min(i0 + b * nthr, total - 1);
      const int row = item >= nb ? 1 : 0;
      const int j = item - row * nb;
      const float2* __restrict__ sp = row ? src1 : src0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        x[b][q] = sp[j + q * nb];
        dd[b][q] = deap[j + q * nb];
      }
    }
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
      const int item = i0 + b * nthr;
      if (item < total) {
        const int row = item >= nb ? 1 : 0;
        const int j = item - row * nb;
        float2 v[8];
        // depths j, j + nb, j + 2nb, j + 3nb sit at r = 6, 7, 0, 1
        dft8_edges<false>(cscale(x[b][2], dd[b][2]), cscale(x[b][3], dd[b][3]), cscale(x[b][0], dd[b][0]),
                          cscale(x[b][1], dd[b][1]), v);
        float2* dst = buf + row * rowstride;
#pragma unroll
        for (int r = 0; r < 8; ++r) dst[fft_swz(j * 8 + r)] = v[r];   // the layout a first radix-8 stage leaves
      }
    }
  }
  __syncthreads();
  fft_ct_stage_range<N, 1, HalfBand<N>::P.ns, MAXB, false>(buf, nrows, rowstride, d, tw, tid, nthr);
}

// Inverse K-point transforms of the LDS rows, stored deapodised as depth
// columns dst0 (row 0) and dst1 (row 1; nullptr: not stored).
template <int N, int MAXB>
__device__ __forceinline__ void adj_grid_ifft_half(float2* buf, int nrows, int rowstride, float2* __restrict__ dst0,
                                                   float2* __restrict__ dst1, const float* __restrict__ deap, int nc,
                                                   const FftDesc& d, const float2* __restrict__ tw, int tid,
                                                   int nthr) {
  using HB = HalfBand<N>;
  constexpr int S = HB::P.ns - 1;
  static_assert(!ct_swz2_out<N, S - 1>(), "the last stage reads the natural layout");
  constexpr int R = HB::RL;
  constexpr int nb = N / R;   // butterflies per row = the stride of the outputs
  constexpr int NQ = fft_tw_pad(R) / 2;
  constexpr int RO = R / 4;   // outputs r < RO and r >= R - RO hold depths
  fft_ct_stage_range<N, 0, S, MAXB, true>(buf, nrows, rowstride, d, tw, tid, nthr);
  const float4* __restrict__ tws = reinterpret_cast<const float4*>(tw + d.tw_off[S]);
  const int total = nrows * nb;
  for (int i0 = tid; i0 < total; i0 += MAXB * nthr) {
    float2 v[MAXB][R];
    float4 wq[MAXB][NQ];
    float dd[MAXB][2 * RO];
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
      const int item = min(i0 + b * nthr, total - 1);
      const int row = item >= nb ? 1 : 0;
      const int k = item - row * nb;
#pragma unroll
      for (int q = 0; q < NQ; ++q) wq[b][q] = tws[k * NQ + q];
#pragma unroll
      for (int r = 0; r < RO; ++r) {
        dd[b][r] = deap[k + r * nb + nc];
        dd[b][RO + r] = deap[k + r * nb];
      }
      const float2* src = buf + row * rowstride + k;
#pragma unroll
      for (int r = 0; r < R; ++r) v[b][r] = src[r * nb];
    }
#pragma unroll
    for (int b = 0; b < MAXB; ++b) {
      const int item = i0 + b * nthr;
      if (item < total) {
        const int row = item >= nb ? 1 : 0;
        const int k = item - row * nb;
        float2* __restrict__ dst = row ? dst1 : dst0;
        if (dst) {
#pragma unroll
          for (int r = 1; r < R; ++r) {
            const float4 q = wq[b][(r - 1) >> 1];
            const float2 w = ((r - 1) & 1) ? make_float2(q.z, -q.w) : make_float2(q.x, -q.y);
            v[b][r] = cmul(v[b][r], w);
          }
          Dft<R, true>::run(v[b]);
          // cell k + r nb: depth k + r nb + n_c for r < RO, k + (r - R + RO) nb for r >= R - RO
#pragma unroll
          for (int r = 0; r < RO; ++r) {
            dst[k + r * nb + nc] = cscale(v[b][r], dd[b][r]);
            dst[k + r * nb] = cscale(v[b][R - RO + r], dd[b][RO + r]);
          }
        }
      }
    }
  }
}

// the half-band forward transform for a compile-time K in SIZES, if there is one
template <int MAXB, int... SIZES>
__device__ __forceinline__ bool fwd_grid_fft_half_sized(float2* buf, int nrows, int rowstride, const float2* src0,
                                                        const float2* src1, const float* deap, const FftDesc& d,
                                                        const float2* tw, int tid, int nthr) {
  bool done = false;
  ((!done && d.n == SIZES && HalfBand<SIZES>::ok
        ? (fwd_grid_fft_half<SIZES, MAXB>(buf, nrows, rowstride, src0, src1, deap, d, tw, tid, nthr), done = true)
        : false),
   ...);
  return done;
}

template <int MAXB, int... SIZES>
__device__ __forceinline__ bool adj_grid_ifft_half_sized(float2* buf, int nrows, int rowstride, float2* dst0,
                                                         float2* dst1, const float* deap, int nc, const FftDesc& d,
                                                         const float2* tw, int tid, int nthr) {
  bool done = false;
  ((!done && d.n == SIZES && HalfBand<SIZES>::ok
        ? (adj_grid_ifft_half<SIZES, MAXB>(buf, nrows, rowstride, dst0, dst1, deap, nc, d, tw, tid, nthr),
           done = true)
        : false),
   ...);
  return done;
}

// element offset of image-side column `lat` (lateral index y n_x + x) of batch item b
__device__ __forceinline__ int64_t xcol(const NufftArgs& a, int b, int lat) {
  const int y = lat / a.Nx, x = lat - y * a.Nx;
  return ((int64_t)(b * (a.Nlat / a.Nx) + y) * a.xs + x) * a.Nz;
}

// per-element loads gathered for batched_for (grid loads and stores; the
// sample loops are not batched: their bodies are long, other waves cover the
// table loads, and batching them would cost registers)
struct VD {
  float2 v;
  float d;
};
struct KP {
  double k2;
  float2 ph;
};
struct KPR {
  double k2;
  float2 ph, r;
};
struct VD2 {
  float2 a, b;
  float d;
};

template <int J, bool ONE>
__global__ void __launch_bounds__(1024) nufft_fwd_kernel(NufftArgs a, const float2* __restrict__ X1,
                                                         float2* __restrict__ W) {
  extern __shared__ float2 gridp[];
  float2* grid = gridp + KPAD;   // cells [-KPAD, K + KPAD)
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int col = blockIdx.x;
  const int lat = col % a.Nlat;
  const int K = a.K, Nz = a.Nz, nc = a.nc;
  const float2* __restrict__ src = X1 + xcol(a, col / a.Nlat, lat);
  const float2* __restrict__ twl = a.twK;

  const bool half = K == 2 * Nz && 2 * nc == Nz &&
                    fwd_grid_fft_half_sized<FftCfg<ONE>::MAXB, OCT_CT_K_SIZES>(grid, 1, K, src, src, a.deap, a.fK,
                                                                                twl, tid, nthr);
  if (!half) {
    // n' = n - n_c placed at n' mod K; cells [Nz - nc, K - nc) stay zero.
    for (int i = tid; i < K - Nz; i += nthr) grid[Nz - nc + i] = make_float2(0.f, 0.f);
    batched_for(Nz, tid, nthr, [&](int n) { return VD{src[n], a.deap[n]}; },
                [&](int n, VD v) {
                  int idx = n - nc;
                  if (idx < 0) idx += K;
                  grid[idx] = cscale(v.v, v.d);
                });
    __syncthreads();
    fft_rows_sized<ONE, false, OCT_CT_K_SIZES>(grid, 1, K, a.fK, twl, tid, nthr);
  }
  if (tid < 2 * KPAD) {   // cells -KPAD..-1 and K..K+KPAD-1 (K >= 2J >= KPAD)
    const int c = tid < KPAD ? tid - KPAD : K + tid - KPAD;
    grid[c] = grid[tid < KPAD ? c + K : c - K];
  }
  __syncthreads();

  const double q2 = a.q2[lat];
  const float bq = a.beam[lat];
  float2* __restrict__ out = W + (int64_t)col * a.Mk;
  for (int m = tid; m < a.Mk; m += nthr) {
    const KP kp{a.k2x4[m], a.phase[m]};
    const double arg = kp.k2 - q2;
    float2 res = make_float2(0.f, 0.f);
    if (arg > 0.0) {
      const double beta = beta_of(arg);
      const double t = a.ct * beta;
      // t mod K (exact: the product is an integer and the difference is
      // representable; a misrounded quotient leaves it one ulp outside [0, K),
      // which the pads absorb); frac(t mod K) = frac(t)
      const double tw = fma(-(double)K, floor(t * a.invK), t);
      const double fl = floor(tw);
      const float x = (float)(2.0 * (tw - fl) - 1.0);
      const int c0 = (int)fl - J / 2 + 1;   // in [-J/2, K - J/2 + 1]
      float2 acc = make_float2(0.f, 0.f);
      const float x2 = x * x;
#pragma unroll
      for (int jj = 0; jj < J / 2; ++jj) {
        float wlo, whi;
        kb_pair(a.kbc + jj * 2 * KBH, x, x2, wlo, whi);
        const float2 g0 = grid[c0 + jj], g1 = grid[c0 + J - 1 - jj];
        acc.x = fmaf(wlo, g0.x, acc.x);
        acc.y = fmaf(wlo, g0.y, acc.y);
        acc.x = fmaf(whi, g1.x, acc.x);
        acc.y = fmaf(whi, g1.y, acc.y);
      }
      res = cmul(filter_h(a, kp.ph, bq, beta), acc);
    }
    out[m] = res;
  }
}

constexpr int EVANESCENT = -(1 << 29);
constexpr short EVANESCENT16 = -32768;

// LDS layout of the adjoint: the sample arrays (filtered samples, tap
// fractions, base cells) and, after the gather, the K-cell grid share one
// region; each thread holds its cells in registers in between.
constexpr int ADJ_MAXC = 8;   // grid cells per thread
constexpr int ADJ_REG_SAMPLES = 2;   // samples per thread kept in registers by the pair adjoint's scatter path

template <int J, bool ONE>
__global__ void __launch_bounds__(1024, ONE ? 8 : 4) nufft_adj_kernel(NufftArgs a, const float2* __restrict__ Rh,
                                                        float2* __restrict__ X) {
  extern __shared__ float4 smem4[];
  __shared__ float kc[J * KBH];
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int col = blockIdx.x;
  const int lat = col % a.Nlat;
  const int K = a.K, Mk = a.Mk, Nz = a.Nz, nc = a.nc;
  const float2* __restrict__ twl = a.twK;
  float2* region = reinterpret_cast<float2*>(smem4);
  float2* grid = region;                    // after the gather
  float2* us = region;                      // before: [Mk] samples
  float* xm = reinterpret_cast<float*>(us + Mk);
  short* bm = reinterpret_cast<short*>(xm + Mk);
  short* first = bm + Mk;                   // [K] first contributing sample of each cell

  // first propagating sample (the evanescent ones form a prefix: lowest k),
  // written by that sample alone; Mk when there is none
  __shared__ int s_mf;
  if (tid == 0) s_mf = Mk;
  for (int i = tid; i < J * KBH; i += nthr) kc[i] = a.kbc[i];
  const double q2 = a.q2[lat];
  const float bq = a.beam[lat];
  const float2* __restrict__ rin = Rh + (int64_t)col * Mk;
  __syncthreads();
  for (int m = tid; m < Mk; m += nthr) {
    const KPR v{a.k2x4[m], a.phase[m], rin[m]};
    const double arg = v.k2 - q2;
    if (arg > 0.0 && (m == 0 || a.k2x4[m - 1] - q2 <= 0.0)) s_mf = m;
    if (arg > 0.0) {
      const double beta = beta_of(arg);
      const double t = a.ct * beta;
      const double fl = floor(t);
      bm[m] = (short)(int)fl;               // t < 32000 (checked at plan creation)
      xm[m] = (float)(2.0 * (t - fl) - 1.0);
      us[m] = cmul(cconj(filter_h(a, v.ph, bq, beta)), v.r);
    } else {
      bm[m] = EVANESCENT16;
      xm[m] = 0.f;
      us[m] = make_float2(0.f, 0.f);
    }
  }
  __syncthreads();

  const int mf = s_mf;
  int umin = 0, umax = -1;
  if (mf < Mk) {
    umin = bm[mf] - J / 2 + 1;
    umax = bm[Mk - 1] + J / 2;
  }
  const int span = umax - umin + 1;
  const int nph = span > K ? (span + K - 1) / K : 1;
  // One phase (the usual case): the first contributor of cell u is the
  // smallest m with bm[m] >= u - J/2, i.e. sample m is first exactly for
  // u in (bm[m-1] + J/2, bm[m] + J/2]; scatter those ranges (they partition
  // the cells, so every entry is written once).
  if (nph == 1) {
    for (int m = mf + tid; m < Mk; m += nthr) {
      const int ulo = (m == mf) ? umin : bm[m - 1] + J / 2 + 1;
      const int uhi = bm[m] + J / 2;
      for (int u = ulo; u <= uhi; ++u) first[u - umin] = (short)m;
    }
    __syncthreads();
  }
  // thread's cells: u = umin + tid + i nthr (+ ph K), i < ADJ_MAXC; grid cell u mod K
  float2 acc[ADJ_MAXC];
#pragma unroll
  for (int i = 0; i < ADJ_MAXC; ++i) acc[i] = make_float2(0.f, 0.f);
  for (int ph = 0; ph < nph; ++ph) {
    const int pbeg = umin + ph * K;
    int pend = pbeg + K;
    if (ph > 0) pend = min(pend, umax + 1);
#pragma unroll
    for (int i = 0; i < ADJ_MAXC; ++i) {
      const int u = pbeg + tid + i * nthr;
      if (u < pend) {
        const int key = u - J / 2;   // first contributor: smallest m with bm[m] >= key
        if (nph == 1) {
          if (u <= umax) {   // cells past umax have no samples
            const int c = u - umin;
            short F[J + 1];
#pragma unroll
            for (int q = 0; q <= J; ++q) F[q] = (c + q < span) ? first[c + q] : (short)Mk;
            float2 sacc = acc[i];
            adj_cell_taps<J, 0>(a.kbc, F, xm, us, sacc);
            acc[i] = sacc;
          }
          continue;
        }
        int p = mf;
        if (mf < Mk) {
          // invert t = ct sqrt(4 k^2 - q^2) for the starting sample, then walk
          // to the exact boundary on the stored base cells
          const double bta = fmax((double)key, 0.0) / a.ct;
          const double km = 0.5 * sqrt(bta * bta + q2);
          double mstar = floor((km - a.k_min) / a.dk);
          mstar = fmin(fmax(mstar, (double)mf), (double)Mk);
          p = (int)mstar;
          while (p > mf && bm[p - 1] >= key) --p;
          while (p < Mk && bm[p] < key) ++p;
        }
        float2 s = acc[i];
        for (int m = p; m < Mk && bm[m] <= u + J / 2 - 1; ++m) {
          const int j = u - (bm[m] - J / 2 + 1);
          const float w = kb_tap<J>(kc, j, xm[m]);
          const float2 uv = us[m];
          s.x = fmaf(w, uv.x, s.x);
          s.y = fmaf(w, uv.y, s.y);
        }
        acc[i] = s;
      }
    }
  }
  __syncthreads();   // sample arrays are dead from here: the grid takes their place
  int g0 = umin % K;   // grid cell of u = umin; the thread's cells follow it
  if (g0 < 0) g0 += K;
#pragma unroll
  for (int i = 0; i < ADJ_MAXC; ++i) {
    if (tid + i * nthr < K) {
      int g = g0 + tid + i * nthr;
      if (g >= K) g -= K;
      grid[g] = acc[i];
    }
  }
  __syncthreads();

  float2* __restrict__ dst = X + xcol(a, col / a.Nlat, lat);
  if (K == 2 * Nz && 2 * nc == Nz &&
      adj_grid_ifft_half_sized<FftCfg<ONE>::MAXB, OCT_CT_K_SIZES>(grid, 1, K, dst, nullptr, a.deap, nc, a.fK, twl,
                                                                   tid, nthr))
    return;
  fft_rows_sized<ONE, true, OCT_CT_K_SIZES>(grid, 1, K, a.fK, twl, tid, nthr);
  batched_for(Nz, tid, nthr, [&](int n) { return a.deap[n]; }, [&](int n, float d) {
    int idx = n - nc;
    if (idx < 0) idx += K;
    dst[n] = cscale(grid[idx], d);
  });
}

// ---------------------------------------------------------------------------
// Half-spectrum column pairs.  Only Re F_lat^{-1} W reaches the measurements
// (eq. (7)), and Re F^{-1} W = F^{-1} W_h with the Hermitian part
// W_h(q) = (W(q) + conj W(-q)) / 2, so W_h is kept for the lateral
// frequencies of one half-plane only.  Columns q and -q have the same |q|^2,
// hence the same beta_m(q), grid coordinates, KB weights and filter: one
// workgroup takes both, forms those once per sample, and runs the two K-point
// transforms as one two-row pass.  The adjoint reads R^(q) once: the residual
// is real, so R^(-q) = conj R^(q), and both image columns come out of one
// gather (one weight evaluation per cell-sample pair for the two columns).
// ---------------------------------------------------------------------------
//
// RES: every measurement pixel observed (s = 1).  Then the lateral round trip
// of the residual, F_lat(Re F_lat^{-1} W - y) / N_lat, is W_h(q) / N_lat -
// Y_h(q) with Y_h = F_lat(y) / N_lat (y is real), so the kernel stores the
// residual spectrum R^ directly (Y_h from r.yh, which may be Wh itself: each
// element is read, then written, by one thread; NULL means y = 0) and, when
// r.partial is set, writes the block's share of ||r||^2 by Parseval:
// sum_l r_l^2 = N_lat sum_q |R^(q)|^2, the pair standing for q and -q.
template <int J, bool ONE, bool RES>
__global__ void __launch_bounds__(1024) nufft_fwd_pair_kernel(NufftArgs a, const float2* __restrict__ X1,
                                                              float2* __restrict__ Wh, PairRes r) {
  extern __shared__ float2 gridp[];
  const int K = a.K, Nz = a.Nz, nc = a.nc;
  const int rs = K + 2 * KPAD;   // row stride: [KPAD pads | K cells | KPAD pads]
  float2* g0 = gridp + KPAD;
  float2* g1 = g0 + rs;
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int b = blockIdx.x / a.n_pairs;
  const int4 pr = a.pairs[blockIdx.x - b * a.n_pairs];
  const float2* __restrict__ s0 = X1 + xcol(a, b, pr.x);
  const float2* __restrict__ s1 = X1 + xcol(a, b, pr.y);
  const int64_t slot = ((int64_t)b * a.n_half + pr.z) * a.Mk;
  // Y_h of this thread's first four samples, loaded before the transforms;
  // each later sample's is loaded four samples ahead (a register ring)
  const float2* yh = RES && r.yh ? r.yh + slot : nullptr;
  auto yload = [&](int m) { return (yh && m < a.Mk) ? yh[m] : make_float2(0.f, 0.f); };
  float2 y0{}, y1{}, y2{}, y3{};
  if constexpr (RES) {
    y0 = yload(tid);
    y1 = yload(tid + nthr);
    y2 = yload(tid + 2 * nthr);
    y3 = yload(tid + 3 * nthr);
  }

  const bool half = K == 2 * Nz && 2 * nc == Nz &&
                    fwd_grid_fft_half_sized<FftCfg<ONE>::MAXB, OCT_CT_K_SIZES>(g0, 2, rs, s0, s1, a.deap, a.fK,
                                                                                a.twK, tid, nthr);
  if (!half) {
    // n' = n - n_c placed at n' mod K; cells [Nz - nc, K - nc) stay zero
    for (int i = tid; i < K - Nz; i += nthr) {
      g0[Nz - nc + i] = make_float2(0.f, 0.f);
      g1[Nz - nc + i] = make_float2(0.f, 0.f);
    }
    batched_for(Nz, tid, nthr, [&](int n) { return VD2{s0[n], s1[n], a.deap[n]}; },
                [&](int n, VD2 v) {
                  int idx = n - nc;
                  if (idx < 0) idx += K;
                  g0[idx] = cscale(v.a, v.d);
                  g1[idx] = cscale(v.b, v.d);
                });
    __syncthreads();
    fft_rows_sized<ONE, false, OCT_CT_K_SIZES>(g0, 2, rs, a.fK, a.twK, tid, nthr);
  }
  if (tid < 4 * KPAD) {   // wrapped copies, cells -KPAD..-1 and K..K+KPAD-1 of both rows
    float2* g = tid < 2 * KPAD ? g0 : g1;
    const int t = tid & (2 * KPAD - 1);
    const int c = t < KPAD ? t - KPAD : K + t - KPAD;
    g[c] = g[t < KPAD ? c + K : c - K];
  }
  __syncthreads();

  const double q2 = a.q2[pr.x];
  const float bq = a.beam[pr.x];
  float2* __restrict__ out = Wh + slot;
  float2* __restrict__ outp = pr.w >= 0 ? Wh + ((int64_t)b * a.n_half + pr.w) * a.Mk : nullptr;
  double acc = 0.0;
  for (int m = tid; m < a.Mk; m += nthr) {
    const KP kp{a.k2x4[m], a.phase[m]};
    const double arg = kp.k2 - q2;
    float2 res = make_float2(0.f, 0.f);
    if (arg > 0.0) {
      const double beta = beta_of(arg);
      const double t = a.ct * beta;
      const double tw = fma(-(double)K, floor(t * a.invK), t);
      const double fl = floor(tw);
      const float x = (float)(2.0 * (tw - fl) - 1.0);
      const int c0 = (int)fl - J / 2 + 1;
      float2 u0 = make_float2(0.f, 0.f), u1 = make_float2(0.f, 0.f);
      const float x2 = x * x;
#pragma unroll
      for (int jj = 0; jj < J / 2; ++jj) {
        float wlo, whi;
        kb_pair(a.kbc + jj * 2 * KBH, x, x2, wlo, whi);
        const float2 a0 = g0[c0 + jj], a1 = g0[c0 + J - 1 - jj];
        const float2 b0 = g1[c0 + jj], b1 = g1[c0 + J - 1 - jj];
        u0.x = fmaf(wlo, a0.x, u0.x);
        u0.y = fmaf(wlo, a0.y, u0.y);
        u0.x = fmaf(whi, a1.x, u0.x);
        u0.y = fmaf(whi, a1.y, u0.y);
        u1.x = fmaf(wlo, b0.x, u1.x);
        u1.y = fmaf(wlo, b0.y, u1.y);
        u1.x = fmaf(whi, b1.x, u1.x);
        u1.y = fmaf(whi, b1.y, u1.y);
      }
      const float2 h = filter_h(a, kp.ph, bq, beta);
      const float2 w0 = cmul(h, u0), w1 = cmul(h, u1);
      res = make_float2(0.5f * (w0.x + w1.x), 0.5f * (w0.y - w1.y));   // (W(q) + conj W(-q)) / 2
    }
    if constexpr (RES) {
      const float2 yv = y0;
      y0 = y1;
      y1 = y2;
      y2 = y3;
      y3 = yload(m + 4 * nthr);
      res = make_float2(fmaf(res.x, r.inv_nlat, -yv.x), fmaf(res.y, r.inv_nlat, -yv.y));
      acc = fma((double)res.x, (double)res.x, fma((double)res.y, (double)res.y, acc));
    }
    out[m] = res;
    if (outp) outp[m] = cconj(res);
  }
  if constexpr (RES) {
    if (r.partial) {   // uniform: every thread takes part in the block sum
      __shared__ double sh[16];
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
      if ((tid & 63) == 0) sh[tid >> 6] = acc;
      __syncthreads();
      if (tid == 0) {
        double t = 0.0;
        for (int w = 0; w < (nthr + 63) >> 6; ++w) t += sh[w];
        r.partial[blockIdx.x] = t * r.nlat * (pr.x != pr.y ? 2.0 : 1.0);
      }
    }
  }
}

// The cell gather of the pair adjoint (the general path): first-contributor
// table, per-cell sums over the samples in increasing m (both columns from one
// weight evaluation), then the sums into the two grid rows.  The sample
// arrays are read from LDS; the grid rows overwrite them at the end.
template <int J>
__device__ __forceinline__ void adj_pair_gather(const NufftArgs& a, const float* kc, double q2, const short* bm,
                                                const float* xm, const float2* us0, const float2* us1, short* first,
                                                float2* grid, int mf, int umin, int umax, int span, int nph,
                                                int tid, int nthr) {
  const int K = a.K, Mk = a.Mk;
  if (nph == 1) {
    for (int m = mf + tid; m < Mk; m += nthr) {
      const int ulo = (m == mf) ? umin : bm[m - 1] + J / 2 + 1;
      const int uhi = bm[m] + J / 2;
      for (int u = ulo; u <= uhi; ++u) first[u - umin] = (short)m;
    }
    __syncthreads();
  }
  float2 acc0[ADJ_MAXC], acc1[ADJ_MAXC];
#pragma unroll
  for (int i = 0; i < ADJ_MAXC; ++i) {
    acc0[i] = make_float2(0.f, 0.f);
    acc1[i] = make_float2(0.f, 0.f);
  }
  for (int ph = 0; ph < nph; ++ph) {
    const int pbeg = umin + ph * K;
    int pend = pbeg + K;
    if (ph > 0) pend = min(pend, umax + 1);
#pragma unroll
    for (int i = 0; i < ADJ_MAXC; ++i) {
      const int u = pbeg + tid + i * nthr;
      if (u < pend) {
        const int key = u - J / 2;
        if (nph == 1) {
          if (u <= umax) {
            const int c = u - umin;
            short F[J + 1];
#pragma unroll
            for (int q = 0; q <= J; ++q) F[q] = (c + q < span) ? first[c + q] : (short)Mk;
            float2 t0 = acc0[i], t1 = acc1[i];
            adj_cell_taps2<J, 0>(a.kbc, F, xm, us0, us1, t0, t1);
            acc0[i] = t0;
            acc1[i] = t1;
          }
          continue;
        }
        int p = mf;
        if (mf < Mk) {
          const double bta = fmax((double)key, 0.0) / a.ct;
          const double km = 0.5 * sqrt(bta * bta + q2);
          double mstar = floor((km - a.k_min) / a.dk);
          mstar = fmin(fmax(mstar, (double)mf), (double)Mk);
          p = (int)mstar;
          while (p > mf && bm[p - 1] >= key) --p;
          while (p < Mk && bm[p] < key) ++p;
        }
        float2 t0 = acc0[i], t1 = acc1[i];
        for (int m = p; m < Mk && bm[m] <= u + J / 2 - 1; ++m) {
          const int j = u - (bm[m] - J / 2 + 1);
          const float w = kb_tap<J>(kc, j, xm[m]);
          const float2 u0 = us0[m], u1 = us1[m];
          t0.x = fmaf(w, u0.x, t0.x);
          t0.y = fmaf(w, u0.y, t0.y);
          t1.x = fmaf(w, u1.x, t1.x);
          t1.y = fmaf(w, u1.y, t1.y);
        }
        acc0[i] = t0;
        acc1[i] = t1;
      }
    }
  }
  __syncthreads();   // sample arrays are dead from here: the two grid rows take their place
  int g0 = umin % K;
  if (g0 < 0) g0 += K;
#pragma unroll
  for (int i = 0; i < ADJ_MAXC; ++i) {
    if (tid + i * nthr < K) {
      int g = g0 + tid + i * nthr;
      if (g >= K) g -= K;
      grid[g] = acc0[i];
      grid[K + g] = acc1[i];
    }
  }
  __syncthreads();

}

template <int J, bool ONE>
__global__ void __launch_bounds__(1024, ONE ? 8 : 4) nufft_adj_pair_kernel(NufftArgs a, const float2* __restrict__ Rh,
                                                                           float2* __restrict__ X) {
  extern __shared__ float4 smem4[];
  __shared__ float kc[J * KBH];
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int K = a.K, Mk = a.Mk, Nz = a.Nz, nc = a.nc;
  const int b = blockIdx.x / a.n_pairs;
  const int4 pr = a.pairs[blockIdx.x - b * a.n_pairs];
  float2* region = reinterpret_cast<float2*>(smem4);
  float2* grid = region;                    // after the gather: two rows of K cells
  float2* us0 = region;                     // before: filtered samples of column q
  float2* us1 = us0 + Mk;                   // and of column -q
  float* xm = reinterpret_cast<float*>(us1 + Mk);
  short* bm = reinterpret_cast<short*>(xm + Mk);
  short* first = bm + Mk;                   // [K] first contributing sample of each cell

  __shared__ int s_mf, s_dup;
  if (tid == 0) {
    s_mf = Mk;
    s_dup = 0;
  }
  for (int i = tid; i < J * KBH; i += nthr) kc[i] = a.kbc[i];
  const double q2 = a.q2[pr.x];
  const float bq = a.beam[pr.x];
  const float2* __restrict__ rin = Rh + ((int64_t)b * a.n_half + pr.z) * Mk;
  __syncthreads();
  // Per-sample setup.  When every thread's samples fit ADJ_REG_SAMPLES, they
  // stay in registers (only the base cells go to LDS, for the checks below);
  // otherwise all sample arrays go to LDS for the cell gather.
  const bool regs = Mk <= ADJ_REG_SAMPLES * nthr;
  int cb[ADJ_REG_SAMPLES];
  float xr[ADJ_REG_SAMPLES];
  float2 u0r[ADJ_REG_SAMPLES], u1r[ADJ_REG_SAMPLES];
  auto setup = [&](int m, int& c, float& x, float2& u0, float2& u1) __attribute__((always_inline)) {
    const KPR v{a.k2x4[m], a.phase[m], rin[m]};
    const double arg = v.k2 - q2;
    if (arg > 0.0 && (m == 0 || a.k2x4[m - 1] - q2 <= 0.0)) s_mf = m;
    if (arg > 0.0) {
      const double beta = beta_of(arg);
      const double t = a.ct * beta;
      const double fl = floor(t);
      c = (int)fl;
      x = (float)(2.0 * (t - fl) - 1.0);
      const float2 hc = cconj(filter_h(a, v.ph, bq, beta));
      u0 = cmul(hc, v.r);
      u1 = cmul(hc, cconj(v.r));
    } else {
      c = EVANESCENT;
      x = 0.f;
      u0 = make_float2(0.f, 0.f);
      u1 = make_float2(0.f, 0.f);
    }
    bm[m] = c == EVANESCENT ? EVANESCENT16 : (short)c;   // t < 32000 (checked at plan creation)
  };
  if (regs) {
#pragma unroll
    for (int i = 0; i < ADJ_REG_SAMPLES; ++i) {
      const int m = tid + i * nthr;
      cb[i] = EVANESCENT;
      xr[i] = 0.f;
      u0r[i] = u1r[i] = make_float2(0.f, 0.f);
      if (m < Mk) setup(m, cb[i], xr[i], u0r[i], u1r[i]);
    }
  } else {
    for (int m = tid; m < Mk; m += nthr) {
      int c;
      float x;
      float2 u0, u1;
      setup(m, c, x, u0, u1);
      xm[m] = x;
      us0[m] = u0;
      us1[m] = u1;
    }
  }
  __syncthreads();

  const int mf = s_mf;
  int umin = 0, umax = -1;
  if (mf < Mk) {
    umin = bm[mf] - J / 2 + 1;
    umax = bm[Mk - 1] + J / 2;
  }
  const int span = umax - umin + 1;
  const int nph = span > K ? (span + K - 1) / K : 1;

  // Scatter path: with distinct base cells (consecutive samples at least a
  // cell apart: sigma >= 2, up to rounding, which the check below catches)
  // and a span within K cells, tap j of every sample hits a different grid
  // cell, so one LDS pass per tap adds w_j u into the cells with no
  // conflicts.  Taps go from J - 1 down to 0, i.e. each cell receives its
  // samples in increasing m: the order of the cell gather.
  if (regs && nph == 1) {
#pragma unroll
    for (int i = 0; i < ADJ_REG_SAMPLES; ++i) {
      const int m = tid + i * nthr;
      if (m > mf && m < Mk && bm[m] <= bm[m - 1]) s_dup = 1;
    }
  }
  __syncthreads();
  if (regs && nph == 1 && !s_dup) {
    for (int i = tid; i < 2 * K; i += nthr) grid[i] = make_float2(0.f, 0.f);   // over the base cells: read above
    float w[ADJ_REG_SAMPLES][J];
    int g0[ADJ_REG_SAMPLES];
#pragma unroll
    for (int i = 0; i < ADJ_REG_SAMPLES; ++i) {
      const float x = xr[i], x2 = x * x;
#pragma unroll
      for (int jj = 0; jj < J / 2; ++jj) kb_pair(a.kbc + jj * 2 * KBH, x, x2, w[i][jj], w[i][J - 1 - jj]);
      int g = (cb[i] - J / 2 + 1) % K;
      g0[i] = g < 0 ? g + K : g;
    }
    __syncthreads();
#pragma unroll
    for (int j = J - 1; j >= 0; --j) {
#pragma unroll
      for (int i = 0; i < ADJ_REG_SAMPLES; ++i) {
        const int m = tid + i * nthr;
        if (m >= mf && m < Mk) {
          int g = g0[i] + j;
          if (g >= K) g -= K;
          float2 c0 = grid[g], c1 = grid[K + g];
          c0.x = fmaf(w[i][j], u0r[i].x, c0.x);
          c0.y = fmaf(w[i][j], u0r[i].y, c0.y);
          c1.x = fmaf(w[i][j], u1r[i].x, c1.x);
          c1.y = fmaf(w[i][j], u1r[i].y, c1.y);
          grid[g] = c0;
          grid[K + g] = c1;
        }
      }
      __syncthreads();
    }
  } else {
    if (regs) {   // the gather reads the samples from LDS
#pragma unroll
      for (int i = 0; i < ADJ_REG_SAMPLES; ++i) {
        const int m = tid + i * nthr;
        if (m < Mk) {
          xm[m] = xr[i];
          us0[m] = u0r[i];
          us1[m] = u1r[i];
        }
      }
      __syncthreads();
    }
    adj_pair_gather<J>(a, kc, q2, bm, xm, us0, us1, first, grid, mf, umin, umax, span, nph, tid, nthr);
  }

  float2* __restrict__ d0 = X + xcol(a, b, pr.x);
  float2* __restrict__ d1 = X + xcol(a, b, pr.y);
  const bool two = pr.y != pr.x;
  if (K == 2 * Nz && 2 * nc == Nz &&
      adj_grid_ifft_half_sized<FftCfg<ONE>::MAXB, OCT_CT_K_SIZES>(grid, 2, K, d0, two ? d1 : nullptr, a.deap, nc,
                                                                   a.fK, a.twK, tid, nthr))
    return;
  fft_rows_sized<ONE, true, OCT_CT_K_SIZES>(grid, 2, K, a.fK, a.twK, tid, nthr);
  batched_for(Nz, tid, nthr, [&](int n) { return a.deap[n]; }, [&](int n, float d) {
    int idx = n - nc;
    if (idx < 0) idx += K;
    d0[n] = cscale(grid[idx], d);
    if (two) d1[n] = cscale(grid[K + idx], d);
  });
}

// ---------------------------------------------------------------------------
// Fully observed plans (s = 1): the normal operator's column part for one
// pair in one kernel.  The forward half is nufft_fwd_pair_kernel's (grid
// rows, K-point transforms, J-tap gather, filter, Hermitian part) ending in
// the residual spectrum R^ = W_h / N_lat - Y_h (eq. (2), (7)); R^ then stays
// in registers as the adjoint's input (NS samples per thread): the sample's
// beta, grid coordinate and filter serve both halves, and R^ makes no round
// trip through HBM.  The adjoint half is nufft_adj_pair_kernel's register
// path.  X1 may be X: a pair reads its two columns before it writes them.
// ---------------------------------------------------------------------------
template <int J, bool ONE, int NS>
__global__ void __launch_bounds__(1024) nufft_normal_pair_kernel(NufftArgs a, const float2* X1, PairRes r,
                                                                 float2* X) {
  extern __shared__ float4 smem4[];
  __shared__ float kc[J * KBH];
  __shared__ int s_mf, s_dup;
  __shared__ double sh[16];
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int K = a.K, Mk = a.Mk, Nz = a.Nz, nc = a.nc;
  const int b = blockIdx.x / a.n_pairs;
  const int4 pr = a.pairs[blockIdx.x - b * a.n_pairs];
  const int64_t slot = ((int64_t)b * a.n_half + pr.z) * Mk;
  const float2* yh = r.yh ? r.yh + slot : nullptr;
  float2 yv[NS];
#pragma unroll
  for (int i = 0; i < NS; ++i) {   // loaded before the transforms
    const int m = tid + i * nthr;
    yv[i] = (yh && m < Mk) ? yh[m] : make_float2(0.f, 0.f);
  }
  if (tid == 0) {
    s_mf = Mk;
    s_dup = 0;
  }
  for (int i = tid; i < J * KBH; i += nthr) kc[i] = a.kbc[i];

  float2* region = reinterpret_cast<float2*>(smem4);
  const int rs = K + 2 * KPAD;   // forward: two grid rows with KPAD wrapped cells on each side
  float2* g0 = region + KPAD;
  float2* g1 = g0 + rs;
  const float2* s0 = X1 + xcol(a, b, pr.x);
  const float2* s1 = X1 + xcol(a, b, pr.y);
  const bool half = K == 2 * Nz && 2 * nc == Nz &&
                    fwd_grid_fft_half_sized<FftCfg<ONE>::MAXB, OCT_CT_K_SIZES>(g0, 2, rs, s0, s1, a.deap, a.fK,
                                                                                a.twK, tid, nthr);
  if (!half) {
    for (int i = tid; i < K - Nz; i += nthr) {
      g0[Nz - nc + i] = make_float2(0.f, 0.f);
      g1[Nz - nc + i] = make_float2(0.f, 0.f);
    }
    batched_for(Nz, tid, nthr, [&](int n) { return VD2{s0[n], s1[n], a.deap[n]}; },
                [&](int n, VD2 v) {
                  int idx = n - nc;
                  if (idx < 0) idx += K;
                  g0[idx] = cscale(v.a, v.d);
                  g1[idx] = cscale(v.b, v.d);
                });
    __syncthreads();
    fft_rows_sized<ONE, false, OCT_CT_K_SIZES>(g0, 2, rs, a.fK, a.twK, tid, nthr);
  }
  if (tid < 4 * KPAD) {
    float2* g = tid < 2 * KPAD ? g0 : g1;
    const int t = tid & (2 * KPAD - 1);
    const int c = t < KPAD ? t - KPAD : K + t - KPAD;
    g[c] = g[t < KPAD ? c + K : c - K];
  }
  __syncthreads();

  const double q2 = a.q2[pr.x];
  const float bq = a.beam[pr.x];
  int cb[NS];
  float xr[NS];
  float2 u0r[NS], u1r[NS];
  double acc = 0.0;
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const int m = tid + i * nthr;
    cb[i] = EVANESCENT;
    xr[i] = 0.f;
    u0r[i] = u1r[i] = make_float2(0.f, 0.f);
    if (m < Mk) {
      const KP kp{a.k2x4[m], a.phase[m]};
      const double arg = kp.k2 - q2;
      float2 res = make_float2(0.f, 0.f), hc = make_float2(0.f, 0.f);
      if (arg > 0.0) {
        if (m == 0 || a.k2x4[m - 1] - q2 <= 0.0) s_mf = m;
        const double beta = beta_of(arg);
        const double t = a.ct * beta;
        const double tw = fma(-(double)K, floor(t * a.invK), t);
        const double flw = floor(tw);
        const float x = (float)(2.0 * (tw - flw) - 1.0);
        const int c0 = (int)flw - J / 2 + 1;
        float2 v0 = make_float2(0.f, 0.f), v1 = make_float2(0.f, 0.f);
        const float x2 = x * x;
#pragma unroll
        for (int jj = 0; jj < J / 2; ++jj) {
          float wlo, whi;
          kb_pair(a.kbc + jj * 2 * KBH, x, x2, wlo, whi);
          const float2 a0 = g0[c0 + jj], a1 = g0[c0 + J - 1 - jj];
          const float2 b0 = g1[c0 + jj], b1 = g1[c0 + J - 1 - jj];
          v0.x = fmaf(wlo, a0.x, v0.x);
          v0.y = fmaf(wlo, a0.y, v0.y);
          v0.x = fmaf(whi, a1.x, v0.x);
          v0.y = fmaf(whi, a1.y, v0.y);
          v1.x = fmaf(wlo, b0.x, v1.x);
          v1.y = fmaf(wlo, b0.y, v1.y);
          v1.x = fmaf(whi, b1.x, v1.x);
          v1.y = fmaf(whi, b1.y, v1.y);
        }
        const float2 h = filter_h(a, kp.ph, bq, beta);
        const float2 w0 = cmul(h, v0), w1 = cmul(h, v1);
        res = make_float2(0.5f * (w0.x + w1.x), 0.5f * (w0.y - w1.y));   // (W(q) + conj W(-q)) / 2
        hc = cconj(h);
        const double fl = floor(t);
        cb[i] = (int)fl;
        xr[i] = (float)(2.0 * (t - fl) - 1.0);
      }
      res = make_float2(fmaf(res.x, r.inv_nlat, -yv[i].x), fmaf(res.y, r.inv_nlat, -yv[i].y));
      acc = fma((double)res.x, (double)res.x, fma((double)res.y, (double)res.y, acc));
      if (cb[i] != EVANESCENT) {
        u0r[i] = cmul(hc, res);
        u1r[i] = cmul(hc, cconj(res));
      }
    }
  }
  if (r.partial) {   // uniform
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if ((tid & 63) == 0) sh[tid >> 6] = acc;
  }
  __syncthreads();   // the forward grid is dead: the adjoint's arrays take its place
  if (r.partial && tid == 0) {
    double t = 0.0;
    for (int w = 0; w < (nthr + 63) >> 6; ++w) t += sh[w];
    r.partial[blockIdx.x] = t * r.nlat * (pr.x != pr.y ? 2.0 : 1.0);
  }
  short* bm = reinterpret_cast<short*>(reinterpret_cast<float*>(region + 2 * Mk) + Mk);
#pragma unroll
  for (int i = 0; i < NS; ++i) {
    const int m = tid + i * nthr;
    if (m < Mk) bm[m] = cb[i] == EVANESCENT ? EVANESCENT16 : (short)cb[i];   // t < 32000 (plan creation)
  }
  __syncthreads();
  // from here as in nufft_adj_pair_kernel (its register path, NS samples per thread)
  const bool regs = true;
  float2* grid = region;
  float2* us0 = region;
  float2* us1 = us0 + Mk;
  float* xm = reinterpret_cast<float*>(us1 + Mk);
  short* first = bm + Mk;
  const int mf = s_mf;
  int umin = 0, umax = -1;
  if (mf < Mk) {
    umin = bm[mf] - J / 2 + 1;
    umax = bm[Mk - 1] + J / 2;
  }
  const int span = umax - umin + 1;
  const int nph = span > K ? (span + K - 1) / K : 1;

  // Scatter path: with distinct base cells (consecutive samples at least a
  // cell apart: sigma >= 2, up to rounding, which the check below catches)
  // and a span within K cells, tap j of every sample hits a different grid
  // cell, so one LDS pass per tap adds w_j u into the cells with no
  // conflicts.  Taps go from J - 1 down to 0, i.e. each cell receives its
  // samples in increasing m: the order of the cell gather.
  if (regs && nph == 1) {
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      const int m = tid + i * nthr;
      if (m > mf && m < Mk && bm[m] <= bm[m - 1]) s_dup = 1;
    }
  }
  __syncthreads();
  if (regs && nph == 1 && !s_dup) {
    for (int i = tid; i < 2 * K; i += nthr) grid[i] = make_float2(0.f, 0.f);   // over the base cells: read above
    float w[NS][J];
    int g0[NS];
#pragma unroll
    for (int i = 0; i < NS; ++i) {
      const float x = xr[i], x2 = x * x;
#pragma unroll
      for (int jj = 0; jj < J / 2; ++jj) kb_pair(a.kbc + jj * 2 * KBH, x, x2, w[i][jj], w[i][J - 1 - jj]);
      int g = (cb[i] - J / 2 + 1) % K;
      g0[i] = g < 0 ? g + K : g;
    }
    __syncthreads();
#pragma unroll
    for (int j = J - 1; j >= 0; --j) {
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        const int m = tid + i * nthr;
        if (m >= mf && m < Mk) {
          int g = g0[i] + j;
          if (g >= K) g -= K;
          float2 c0 = grid[g], c1 = grid[K + g];
          c0.x = fmaf(w[i][j], u0r[i].x, c0.x);
          c0.y = fmaf(w[i][j], u0r[i].y, c0.y);
          c1.x = fmaf(w[i][j], u1r[i].x, c1.x);
          c1.y = fmaf(w[i][j], u1r[i].y, c1.y);
          grid[g] = c0;
          grid[K + g] = c1;
        }
      }
      __syncthreads();
    }
  } else {
    if (regs) {   // the gather reads the samples from LDS
#pragma unroll
      for (int i = 0; i < NS; ++i) {
        const int m = tid + i * nthr;
        if (m < Mk) {
          xm[m] = xr[i];
          us0[m] = u0r[i];
          us1[m] = u1r[i];
        }
      }
      __syncthreads();
    }
    adj_pair_gather<J>(a, kc, q2, bm, xm, us0, us1, first, grid, mf, umin, umax, span, nph, tid, nthr);
  }

  float2* __restrict__ d0 = X + xcol(a, b, pr.x);
  float2* __restrict__ d1 = X + xcol(a, b, pr.y);
  const bool two = pr.y != pr.x;
  if (K == 2 * Nz && 2 * nc == Nz &&
      adj_grid_ifft_half_sized<FftCfg<ONE>::MAXB, OCT_CT_K_SIZES>(grid, 2, K, d0, two ? d1 : nullptr, a.deap, nc,
                                                                   a.fK, a.twK, tid, nthr))
    return;
  fft_rows_sized<ONE, true, OCT_CT_K_SIZES>(grid, 2, K, a.fK, a.twK, tid, nthr);
  batched_for(Nz, tid, nthr, [&](int n) { return a.deap[n]; }, [&](int n, float d) {
    int idx = n - nc;
    if (idx < 0) idx += K;
    d0[n] = cscale(grid[idx], d);
    if (two) d1[n] = cscale(grid[K + idx], d);
  });
}


// Threads per column: enough for the FFT stages, and wide enough that the
// per-column work is short (the column count of a B-scan is only ~1000).
int nufft_threads(const NufftArgs& a, int want) {
  const int bf = a.K / a.fK.min_radix;
  const int mb = fft_maxb(a.fK);
  int nt = 256;
  while (nt < 1024 && (bf > mb * nt || nt < want)) nt <<= 1;
  return nt;
}

}  // namespace

size_t nufft_adj_lds_bytes(const NufftArgs& a) {
  const size_t samples = (size_t)a.Mk * (sizeof(float2) + sizeof(float) + sizeof(short)) + (size_t)a.K * sizeof(short);
  const size_t grid = (size_t)a.K * sizeof(float2);
  return samples > grid ? samples : grid;
}

int nufft_adj_threads(const NufftArgs& a) {
  // every thread keeps at most ADJ_MAXC grid cells in registers; with many
  // columns (batches, volumes) narrower groups keep more columns in flight
  // per CU, which hides their barrier-separated phases better
  int nt = nufft_threads(a, a.n_cols >= 4096 ? 256 : 512);
  while (nt < 1024 && (a.K + nt - 1) / nt > ADJ_MAXC) nt <<= 1;
  return nt;
}

template <int J, bool ONE>
hipError_t nufft_fwd_t(const NufftArgs& a, const float2* X1, float2* W, int nthr, hipStream_t s) {
  const size_t lds = (size_t)(a.K + 2 * KPAD) * sizeof(float2);
  if (lds > 64 * 1024) {
    // once per instantiation (thread-safe initialisation of a local static)
    static const hipError_t set = hipFuncSetAttribute(reinterpret_cast<const void*>(&nufft_fwd_kernel<J, ONE>),
                                                      hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 2048);
    if (set != hipSuccess) return set;
  }
  hipLaunchKernelGGL((nufft_fwd_kernel<J, ONE>), dim3(a.n_cols), dim3(nthr), lds, s, a, X1, W);
  return hipGetLastError();
}

hipError_t launch_nufft_fwd(const NufftArgs& a, const float2* X1, float2* W, hipStream_t s) {
  const int nt = nufft_threads(a, 256);
  const bool one = fft_one(a.fK, 1, nt);
  switch (a.J) {
    case 4: return one ? nufft_fwd_t<4, true>(a, X1, W, nt, s) : nufft_fwd_t<4, false>(a, X1, W, nt, s);
    case 6: return one ? nufft_fwd_t<6, true>(a, X1, W, nt, s) : nufft_fwd_t<6, false>(a, X1, W, nt, s);
    default: return one ? nufft_fwd_t<8, true>(a, X1, W, nt, s) : nufft_fwd_t<8, false>(a, X1, W, nt, s);
  }
}

template <int J, bool ONE>
hipError_t nufft_adj_t(const NufftArgs& a, const float2* Rh, float2* X, int nthr, hipStream_t s) {
  const size_t lds = nufft_adj_lds_bytes(a);
  if (lds > 64 * 1024 - 1024) {
    // once per instantiation (thread-safe initialisation of a local static)
    static const hipError_t set = hipFuncSetAttribute(reinterpret_cast<const void*>(&nufft_adj_kernel<J, ONE>),
                                                      hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 2048);
    if (set != hipSuccess) return set;
  }
  hipLaunchKernelGGL((nufft_adj_kernel<J, ONE>), dim3(a.n_cols), dim3(nthr), lds, s, a, Rh, X);
  return hipGetLastError();
}

hipError_t launch_nufft_adj(const NufftArgs& a, const float2* Rh, float2* X, hipStream_t s) {
  const int nt = nufft_adj_threads(a);
  const bool one = fft_one(a.fK, 1, nt);
  switch (a.J) {
    case 4: return one ? nufft_adj_t<4, true>(a, Rh, X, nt, s) : nufft_adj_t<4, false>(a, Rh, X, nt, s);
    case 6: return one ? nufft_adj_t<6, true>(a, Rh, X, nt, s) : nufft_adj_t<6, false>(a, Rh, X, nt, s);
    default: return one ? nufft_adj_t<8, true>(a, Rh, X, nt, s) : nufft_adj_t<8, false>(a, Rh, X, nt, s);
  }
}

// ---- half-spectrum column pairs
size_t nufft_pair_lds_bytes(const NufftArgs& a, bool adjoint) {
  if (!adjoint) return (size_t)2 * (a.K + 2 * KPAD) * sizeof(float2);
  const size_t samples = (size_t)a.Mk * (2 * sizeof(float2) + sizeof(float) + sizeof(short)) + (size_t)a.K * sizeof(short);
  const size_t grid = (size_t)2 * a.K * sizeof(float2);
  return samples > grid ? samples : grid;
}

namespace {

// threads for two K-point rows: every stage's butterflies fit (at most two
// per thread), and the adjoint's cells fit ADJ_MAXC per thread
int pair_threads(const NufftArgs& a, bool adjoint) {
  const int bf = 2 * (a.K / a.fK.min_radix);
  const int mb = fft_maxb(a.fK);
  int nt = adjoint ? 512 : 256;
  while (nt < 1024 && (bf > mb * nt || (adjoint && (a.K + nt - 1) / nt > ADJ_MAXC))) nt <<= 1;
  if (adjoint && nt < 1024 && fft_one(a.fK, 2, 2 * nt) && !fft_one(a.fK, 2, nt)) nt <<= 1;   // one butterfly per thread
  return nt;
}

template <int J, bool ONE, bool RES>
hipError_t nufft_fwd_pair_t(const NufftArgs& a, const float2* X1, float2* Wh, const PairRes& r, int nthr,
                            hipStream_t s) {
  const size_t lds = nufft_pair_lds_bytes(a, false);
  if (lds > 64 * 1024) {
    static const hipError_t set =
        hipFuncSetAttribute(reinterpret_cast<const void*>(&nufft_fwd_pair_kernel<J, ONE, RES>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 2048);
    if (set != hipSuccess) return set;
  }
  hipLaunchKernelGGL((nufft_fwd_pair_kernel<J, ONE, RES>), dim3(a.n_pairs * (a.n_cols / a.Nlat)), dim3(nthr), lds, s,
                     a, X1, Wh, r);
  return hipGetLastError();
}

template <bool RES>
hipError_t fwd_pair_dispatch(const NufftArgs& a, const float2* X1, float2* Wh, const PairRes& r, hipStream_t s) {
  const int nt = pair_threads(a, false);
  const bool one = fft_one(a.fK, 2, nt);
  switch (a.J) {
    case 4: return one ? nufft_fwd_pair_t<4, true, RES>(a, X1, Wh, r, nt, s)
                       : nufft_fwd_pair_t<4, false, RES>(a, X1, Wh, r, nt, s);
    case 6: return one ? nufft_fwd_pair_t<6, true, RES>(a, X1, Wh, r, nt, s)
                       : nufft_fwd_pair_t<6, false, RES>(a, X1, Wh, r, nt, s);
    default: return one ? nufft_fwd_pair_t<8, true, RES>(a, X1, Wh, r, nt, s)
                        : nufft_fwd_pair_t<8, false, RES>(a, X1, Wh, r, nt, s);
  }
}

template <int J, bool ONE>
hipError_t nufft_adj_pair_t(const NufftArgs& a, const float2* Rh, float2* X, int nthr, hipStream_t s) {
  const size_t lds = nufft_pair_lds_bytes(a, true);
  if (lds > 64 * 1024 - 1024) {
    static const hipError_t set = hipFuncSetAttribute(reinterpret_cast<const void*>(&nufft_adj_pair_kernel<J, ONE>),
                                                      hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 2048);
    if (set != hipSuccess) return set;
  }
  hipLaunchKernelGGL((nufft_adj_pair_kernel<J, ONE>), dim3(a.n_pairs * (a.n_cols / a.Nlat)), dim3(nthr), lds, s, a, Rh,
                     X);
  return hipGetLastError();
}

}  // namespace

bool nufft_pair_supported(const NufftArgs& a) {
  constexpr size_t lds_max = 156 * 1024;
  if (nufft_pair_lds_bytes(a, false) > lds_max || nufft_pair_lds_bytes(a, true) > lds_max) return false;
  const int bf = 2 * (a.K / a.fK.min_radix);
  const int mb = fft_maxb(a.fK);
  for (bool adj : {false, true}) {
    const int nt = pair_threads(a, adj);
    if (bf > mb * nt || (adj && (a.K + nt - 1) / nt > ADJ_MAXC)) return false;
  }
  return true;
}

hipError_t launch_nufft_fwd_pair(const NufftArgs& a, const float2* X1, float2* Wh, hipStream_t s) {
  return fwd_pair_dispatch<false>(a, X1, Wh, PairRes{}, s);
}

hipError_t launch_nufft_fwd_pair_res(const NufftArgs& a, const float2* X1, float2* Rh, const float2* yh,
                                     double* partial, hipStream_t s) {
  PairRes r{};
  r.yh = yh;
  r.partial = partial;
  r.inv_nlat = 1.f / (float)a.Nlat;
  r.nlat = (double)a.Nlat;
  return fwd_pair_dispatch<true>(a, X1, Rh, r, s);
}

namespace {
constexpr int NORMAL_NS = 4;   // samples per thread of the fused pair kernel

template <int J, bool ONE>
hipError_t nufft_normal_pair_t(const NufftArgs& a, const float2* X1, const PairRes& r, float2* X, int nthr,
                               hipStream_t s) {
  const size_t lds = nufft_normal_pair_lds_bytes(a);
  if (lds > 64 * 1024 - 1024) {
    static const hipError_t set =
        hipFuncSetAttribute(reinterpret_cast<const void*>(&nufft_normal_pair_kernel<J, ONE, NORMAL_NS>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 2048);
    if (set != hipSuccess) return set;
  }
  hipLaunchKernelGGL((nufft_normal_pair_kernel<J, ONE, NORMAL_NS>), dim3(a.n_pairs * (a.n_cols / a.Nlat)),
                     dim3(nthr), lds, s, a, X1, r, X);
  return hipGetLastError();
}
}  // namespace

size_t nufft_normal_pair_lds_bytes(const NufftArgs& a) {
  const size_t f = nufft_pair_lds_bytes(a, false), g = nufft_pair_lds_bytes(a, true);
  return f > g ? f : g;
}

// the forward kernel's threads; every thread's samples and grid cells fit its registers
bool nufft_normal_pair_supported(const NufftArgs& a) {
  const int nt = pair_threads(a, false);
  return nufft_pair_supported(a) && nufft_normal_pair_lds_bytes(a) <= 156 * 1024 && a.Mk <= NORMAL_NS * nt &&
         (a.K + nt - 1) / nt <= ADJ_MAXC;
}

hipError_t launch_nufft_normal_pair(const NufftArgs& a, const float2* X1, const float2* yh, double* partial,
                                    float2* X, hipStream_t s) {
  const int nt = pair_threads(a, false);
  const bool one = fft_one(a.fK, 2, nt);
  PairRes r{};
  r.yh = yh;
  r.partial = partial;
  r.inv_nlat = 1.f / (float)a.Nlat;
  r.nlat = (double)a.Nlat;
  switch (a.J) {
    case 4: return one ? nufft_normal_pair_t<4, true>(a, X1, r, X, nt, s) : nufft_normal_pair_t<4, false>(a, X1, r, X, nt, s);
    case 6: return one ? nufft_normal_pair_t<6, true>(a, X1, r, X, nt, s) : nufft_normal_pair_t<6, false>(a, X1, r, X, nt, s);
    default: return one ? nufft_normal_pair_t<8, true>(a, X1, r, X, nt, s) : nufft_normal_pair_t<8, false>(a, X1, r, X, nt, s);
  }
}

hipError_t launch_nufft_adj_pair(const NufftArgs& a, const float2* Rh, float2* X, hipStream_t s) {
  const int nt = pair_threads(a, true);
  const bool one = fft_one(a.fK, 2, nt);
  switch (a.J) {
    case 4: return one ? nufft_adj_pair_t<4, true>(a, Rh, X, nt, s) : nufft_adj_pair_t<4, false>(a, Rh, X, nt, s);
    case 6: return one ? nufft_adj_pair_t<6, true>(a, Rh, X, nt, s) : nufft_adj_pair_t<6, false>(a, Rh, X, nt, s);
    default: return one ? nufft_adj_pair_t<8, true>(a, Rh, X, nt, s) : nufft_adj_pair_t<8, false>(a, Rh, X, nt, s);
  }
}
