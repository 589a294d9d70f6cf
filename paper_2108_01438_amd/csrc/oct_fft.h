// In-LDS mixed-radix Stockham FFT (radices 2, 3, 4, 5, 7, 8) for gfx950.
//
// Each stage with radix R and sub-transform size Ns reads butterfly j from
// positions j + r n/R, applies the twiddles w^{r (j mod Ns)} with
// w = e^{-+2 pi i / (Ns R)}, takes a radix-R DFT and writes output r to
// (j div Ns) Ns R + (j mod Ns) + r Ns, which leaves the result in natural
// order (the Stockham autosort formulation of Govindaraju et al., 2008).
// The transform runs in place in one LDS buffer: every thread first pulls
// all of its butterflies into registers, a barrier separates the reads from
// the writes, so the per-stage work must fit MAXB butterflies per thread.
// Twiddles come from per-stage rows in global memory (FP64-built, rounded
// once to FP32): row k of a stage holds w^{r k} for r = 1..R-1, so a
// butterfly fetches its R-1 factors with 16-byte loads through the vector
// cache, issued before the stage's LDS reads so that their latency overlaps
// the barrier.
#pragma once
#include "oct_common.h"

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
// multiply by -i (forward) or +i (inverse)
template <bool INV>
__device__ __forceinline__ float2 rot90(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

__device__ __forceinline__ uint32_t fdiv(uint32_t x, const FastDiv& f) {
  if (f.s < 0) return x;
  const uint32_t t = __umulhi(f.m, x);
  return (t + ((x - t) >> 1)) >> f.s;
}

// LDS bank swizzle between the first two stages of a transform whose first
// radix is 8: the first stage writes butterfly j's outputs to 8j + r, eight
// lanes apart for one r; XOR-ing the low three bits of the index with the
// next three spreads those writes over the banks.  The map only permutes
// indices inside aligned groups of eight (n is a multiple of 8), so the
// second stage, which reads through the same map, sees the same data.
__device__ __forceinline__ int fft_swz(int i) { return i ^ ((i >> 3) & 7); }

// The same for the second radix-8 stage (sub-transform size 8) when a stage
// follows it: butterfly j writes output r to 64 (j div 8) + (j mod 8) + 8 r,
// so for one r the 64 lanes of a wave cover only eight bank pairs.  Flipping
// bit 3 of the index with bit 6 gives each group of 16 lanes 16 distinct bank
// pairs; the map permutes inside aligned groups of 16 and is its own inverse,
// and the next stage reads through it.
__device__ __forceinline__ int fft_swz2(int i) { return i ^ ((i >> 3) & 8); }

// Element loop with batched loads: every thread first issues the loads of U
// elements (indices clamped to a valid element, so each load is in bounds
// and none waits on another), then consumes them in order.  A plain loop
// would wait for each element's load before issuing the next.
template <int U = 8, class Load, class Use>
__device__ __forceinline__ void batched_for(int n, int tid, int nthr, Load load, Use use) {
  using R = decltype(load(0));
  for (int i0 = tid; i0 < n; i0 += U * nthr) {
    R r[U];
#pragma unroll
    for (int u = 0; u < U; ++u) r[u] = load(min(i0 + u * nthr, n - 1));
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i0 + u * nthr < n) use(i0 + u * nthr, r[u]);
  }
}

template <int R, bool INV> struct Dft;

template <bool INV> struct Dft<2, INV> {
  static __device__ __forceinline__ void run(float2* a) {
    float2 t = a[1];
    a[1] = csub(a[0], t);
    a[0] = cadd(a[0], t);
  }
};

template <bool INV> struct Dft<4, INV> {
  static __device__ __forceinline__ void run(float2* a) {
    float2 s0 = cadd(a[0], a[2]), d0 = csub(a[0], a[2]);
    float2 s1 = cadd(a[1], a[3]), d1 = rot90<INV>(csub(a[1], a[3]));
    a[0] = cadd(s0, s1);
    a[2] = csub(s0, s1);
    a[1] = cadd(d0, d1);
    a[3] = csub(d0, d1);
  }
};

template <bool INV> struct Dft<8, INV> {
  static __device__ __forceinline__ void run(float2* a) {
    float2 b[4], c[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      b[k] = cadd(a[k], a[k + 4]);
      c[k] = csub(a[k], a[k + 4]);
    }
    finish(b, c, a);
  }
  // the rest of the DFT from b_k = a_k + a_{k+4} and c_k = a_k - a_{k+4}
  static __device__ __forceinline__ void finish(float2* b, float2* c, float2* a) {
    const float h = 0.70710678118654752440f;
    // c_k *= w8^k, w8 = e^{-+ i pi / 4}
    {
      float2 t = c[1];
      c[1] = INV ? make_float2(h * (t.x - t.y), h * (t.x + t.y))
                 : make_float2(h * (t.x + t.y), h * (t.y - t.x));
      c[2] = rot90<INV>(c[2]);
      t = c[3];
      c[3] = INV ? make_float2(-h * (t.x + t.y), h * (t.x - t.y))
                 : make_float2(h * (t.y - t.x), -h * (t.x + t.y));
    }
    Dft<4, INV>::run(b);
    Dft<4, INV>::run(c);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      a[2 * m] = b[m];
      a[2 * m + 1] = c[m];
    }
  }
};

// Radix 3, 5, 7: direct DFT with compile-time roots of unity.
template <int R> struct Roots;
template <> struct Roots<3> {
  static __device__ __forceinline__ float c(int k) {
    const float v[3] = {1.0f, -0.5f, -0.5f};
    return v[k];
  }
  static __device__ __forceinline__ float s(int k) {
    const float v[3] = {0.0f, 0.86602540378443864676f, -0.86602540378443864676f};
    return v[k];
  }
};
template <> struct Roots<5> {
  static __device__ __forceinline__ float c(int k) {
    const float v[5] = {1.0f, 0.30901699437494742410f, -0.80901699437494742410f,
                        -0.80901699437494742410f, 0.30901699437494742410f};
    return v[k];
  }
  static __device__ __forceinline__ float s(int k) {
    const float v[5] = {0.0f, 0.95105651629515357212f, 0.58778525229247312917f,
                        -0.58778525229247312917f, -0.95105651629515357212f};
    return v[k];
  }
};
template <> struct Roots<7> {
  static __device__ __forceinline__ float c(int k) {
    const float v[7] = {1.0f, 0.62348980185873353053f, -0.22252093395631440429f,
                        -0.90096886790241912624f, -0.90096886790241912624f,
                        -0.22252093395631440429f, 0.62348980185873353053f};
    return v[k];
  }
  static __device__ __forceinline__ float s(int k) {
    const float v[7] = {0.0f, 0.78183148246802980871f, 0.97492791218182360702f,
                        0.43388373911755812048f, -0.43388373911755812048f,
                        -0.97492791218182360702f, -0.78183148246802980871f};
    return v[k];
  }
};

// Odd radix by the pair symmetry of the DFT: with t_r = a_r + a_{R-r} and
// u_r = a_r - a_{R-r} (r = 1..(R-1)/2), X_0 = a_0 + sum t_r and, for
// s = 1..(R-1)/2, X_s = A_s -+ i B_s, X_{R-s} = A_s +- i B_s with
// A_s = a_0 + sum_r cos(2 pi r s / R) t_r, B_s = sum_r sin(2 pi r s / R) u_r.
template <int R, bool INV> struct DftOdd {
  static __device__ __forceinline__ void run(float2* a) {
    constexpr int h = (R - 1) / 2;
    float2 t[h + 1], u[h + 1];
#pragma unroll
    for (int r = 1; r <= h; ++r) {
      t[r] = cadd(a[r], a[R - r]);
      u[r] = csub(a[r], a[R - r]);
    }
    float2 x0 = a[0];
#pragma unroll
    for (int r = 1; r <= h; ++r) x0 = cadd(x0, t[r]);
#pragma unroll
    for (int s = 1; s <= h; ++s) {
      float2 A = a[0], Bv = make_float2(0.f, 0.f);
#pragma unroll
      for (int r = 1; r <= h; ++r) {
        const int k = (r * s) % R;
        const float cr = Roots<R>::c(k), sr = Roots<R>::s(k);
        A.x = fmaf(cr, t[r].x, A.x);
        A.y = fmaf(cr, t[r].y, A.y);
        Bv.x = fmaf(sr, u[r].x, Bv.x);
        Bv.y = fmaf(sr, u[r].y, Bv.y);
      }
      // -i B (forward) or +i B (inverse)
      const float2 iB = rot90<INV>(Bv);
      a[s] = cadd(A, iB);
      a[R - s] = csub(A, iB);
    }
    a[0] = x0;
  }
};
template <bool INV> struct Dft<3, INV> : DftOdd<3, INV> {};
template <bool INV> struct Dft<5, INV> : DftOdd<5, INV> {};
template <bool INV> struct Dft<7, INV> : DftOdd<7, INV> {};

// One Stockham stage over `nrows` transforms of length n stored at
// buf[row * rowstride + i]; tw: this stage's twiddle rows (global memory).
template <int R, int MAXB, bool INV>
__device__ __forceinline__ void fft_stage(float2* buf, int nrows, int rowstride, int n, int Ns,
                                          const FastDiv& dnb, const FastDiv& dns,
                                          const float2* __restrict__ tw, int tid, int nthr) {
  constexpr int NQ = fft_tw_pad(R) / 2;   // 16-byte loads per butterfly
  const int nb = n / R;
  const int total = nrows * nb;
  float2 v[MAXB][R];
  float4 wq[MAXB][NQ];
  int off[MAXB], jj[MAXB], kk[MAXB];
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int item = tid + b * nthr;
    if (item < total) {
      const int row = (int)fdiv((uint32_t)item, dnb);
      const int j = item - row * nb;
      const int k = j - (int)fdiv((uint32_t)j, dns) * Ns;
      if (Ns > 1) {
        const float4* tp = reinterpret_cast<const float4*>(tw) + k * NQ;
#pragma unroll
        for (int q = 0; q < NQ; ++q) wq[b][q] = tp[q];
      }
      const float2* src = buf + row * rowstride;
      if (Ns == 8) {   // second stage after a first radix-8 stage: swizzled layout
#pragma unroll
        for (int r = 0; r < R; ++r) v[b][r] = src[fft_swz(j + r * nb)];
      } else {
#pragma unroll
        for (int r = 0; r < R; ++r) v[b][r] = src[j + r * nb];
      }
      off[b] = row * rowstride;
      jj[b] = j;
      kk[b] = k;
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int item = tid + b * nthr;
    if (item < total) {
      const int j = jj[b], k = kk[b];
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const float4 q = wq[b][(r - 1) >> 1];
          float2 w = ((r - 1) & 1) ? make_float2(q.z, q.w) : make_float2(q.x, q.y);
          if (INV) w.y = -w.y;
          v[b][r] = cmul(v[b][r], w);
        }
      }
      Dft<R, INV>::run(v[b]);
      if (R == 8 && Ns == 1 && n > 8) {   // first stage of several: swizzled layout
        float2* dst = buf + off[b];
#pragma unroll
        for (int r = 0; r < R; ++r) dst[fft_swz(j * R + r)] = v[b][r];
      } else {
        float2* dst = buf + off[b] + (j - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) dst[r * Ns] = v[b][r];
      }
    }
  }
  __syncthreads();
}

// Full transform of `nrows` rows in LDS; all threads of the block participate.
// ONE selects the variant with one butterfly per thread and stage (fewer
// registers); the other variant runs up to two butterflies per thread.
template <bool ONE>
struct FftCfg {
  static constexpr int MAXB = ONE ? 1 : 2;
};

template <bool ONE, bool INV>
__device__ __forceinline__ void fft_rows(float2* buf, int nrows, int rowstride, const FftDesc& d,
                                         const float2* __restrict__ tw, int tid, int nthr) {
  constexpr int MB = FftCfg<ONE>::MAXB;
  for (int s = 0; s < d.nstages; ++s) {
    const int Ns = d.ns[s];
    const float2* t = tw + d.tw_off[s];
    switch (d.radix[s]) {
      case 8: fft_stage<8, MB, INV>(buf, nrows, rowstride, d.n, Ns, d.div_nb[s], d.div_ns[s], t, tid, nthr); break;
      case 4: fft_stage<4, MB, INV>(buf, nrows, rowstride, d.n, Ns, d.div_nb[s], d.div_ns[s], t, tid, nthr); break;
      case 2: fft_stage<2, MB, INV>(buf, nrows, rowstride, d.n, Ns, d.div_nb[s], d.div_ns[s], t, tid, nthr); break;
      case 5: fft_stage<5, MB, INV>(buf, nrows, rowstride, d.n, Ns, d.div_nb[s], d.div_ns[s], t, tid, nthr); break;
      case 3: fft_stage<3, MB, INV>(buf, nrows, rowstride, d.n, Ns, d.div_nb[s], d.div_ns[s], t, tid, nthr); break;
      default: fft_stage<7, MB, INV>(buf, nrows, rowstride, d.n, Ns, d.div_nb[s], d.div_ns[s], t, tid, nthr); break;
    }
  }
}

// ---------------------------------------------------------------------------
// Compile-time transform lengths.  For the lengths a kernel instantiates, the
// radix plan, every stride, the butterfly counts and the k = j mod Ns
// divisions are constants: LDS offsets fold into the instructions (paired
// reads and writes), and the index arithmetic of the generic path disappears.
// The radix plan is the host's (factorize in oct_api.cpp): radix 8 with a 4
// (or 4 x 4) instead of a trailing 2, then 5, 3, 7; the twiddle rows are the
// host's too (offsets from the descriptor).
// ---------------------------------------------------------------------------
struct CtPlan {
  int ns;
  int r[OCT_MAX_STAGES];
};
constexpr CtPlan ct_plan(int n) {
  CtPlan p{};
  int m = n, a = 0;
  while (m % 2 == 0) { m /= 2; ++a; }
  const int q = a / 3, rem = a % 3;
  if (rem == 1 && q >= 1) {
    for (int i = 0; i < q - 1; ++i) p.r[p.ns++] = 8;
    p.r[p.ns++] = 4;
    p.r[p.ns++] = 4;
  } else {
    for (int i = 0; i < q; ++i) p.r[p.ns++] = 8;
    if (rem == 1) p.r[p.ns++] = 2;
    if (rem == 2) p.r[p.ns++] = 4;
  }
  const int odd[3] = {5, 3, 7};
  for (int i = 0; i < 3; ++i)
    while (m % odd[i] == 0) { m /= odd[i]; p.r[p.ns++] = odd[i]; }
  return p;
}
constexpr int ct_ns_before(const CtPlan& p, int s) {
  int v = 1;
  for (int i = 0; i < s; ++i) v *= p.r[i];
  return v;
}

template <int R, int N, int NS, int MAXB, bool INV, bool SWZ2_IN = false, bool SWZ2_OUT = false>
__device__ __forceinline__ void fft_stage_ct(float2* buf, int nrows, int rowstride,
                                             const float2* __restrict__ tw, int tid, int nthr) {
  constexpr int NQ = fft_tw_pad(R) / 2;
  constexpr int nb = N / R;
  const int total = nrows * nb;
  float2 v[MAXB][R];
  float4 wq[MAXB][NQ];
  int base[MAXB], jj[MAXB];
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int item = tid + b * nthr;
    if (item < total) {
      const int row = item / nb;
      const int j = item - row * nb;
      if (NS > 1) {
        const int k = j % NS;
        const float4* tp = reinterpret_cast<const float4*>(tw) + k * NQ;
#pragma unroll
        for (int q = 0; q < NQ; ++q) wq[b][q] = tp[q];
      }
      base[b] = row * rowstride;
      if (NS == 8) {   // second stage after a first radix-8 stage: swizzled layout
        const float2* src = buf + base[b];
#pragma unroll
        for (int r = 0; r < R; ++r) v[b][r] = src[fft_swz(j + r * nb)];
      } else if (SWZ2_IN) {   // after a swizzled second stage
        const float2* src = buf + base[b];
#pragma unroll
        for (int r = 0; r < R; ++r) v[b][r] = src[fft_swz2(j + r * nb)];
      } else {
        const float2* src = buf + base[b] + j;
#pragma unroll
        for (int r = 0; r < R; ++r) v[b][r] = src[r * nb];
      }
      jj[b] = j;
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int item = tid + b * nthr;
    if (item < total) {
      const int j = jj[b], k = j % NS;
      if (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          const float4 q = wq[b][(r - 1) >> 1];
          float2 w = ((r - 1) & 1) ? make_float2(q.z, q.w) : make_float2(q.x, q.y);
          if (INV) w.y = -w.y;
          v[b][r] = cmul(v[b][r], w);
        }
      }
      Dft<R, INV>::run(v[b]);
      if (R == 8 && NS == 1 && N > 8) {   // first stage of several: swizzled layout
        float2* dst = buf + base[b];
#pragma unroll
        for (int r = 0; r < R; ++r) dst[fft_swz(j * R + r)] = v[b][r];
      } else if (SWZ2_OUT) {
        float2* dst = buf + base[b];
        const int o = (j - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) dst[fft_swz2(o + r * NS)] = v[b][r];
      } else {
        float2* dst = buf + base[b] + (j - k) * R + k;
#pragma unroll
        for (int r = 0; r < R; ++r) dst[r * NS] = v[b][r];
      }
    }
  }
  __syncthreads();
}

// Stage S of the plan of length N writes through fft_swz2 when it is a
// radix-8 stage of sub-transform size 8 and another stage follows; stage S
// reads through it when stage S - 1 did.
template <int N, int S>
constexpr bool ct_swz2_out() {
  constexpr CtPlan P = ct_plan(N);
  return S >= 0 && S + 1 < P.ns && P.r[S] == 8 && ct_ns_before(P, S) == 8;
}

// stages S..E-1 of the compile-time plan of length N
template <int N, int S, int E, int MAXB, bool INV>
__device__ __forceinline__ void fft_ct_stage_range(float2* buf, int nrows, int rowstride, const FftDesc& d,
                                                   const float2* __restrict__ tw, int tid, int nthr) {
  constexpr CtPlan P = ct_plan(N);
  if constexpr (S < E) {
    fft_stage_ct<P.r[S], N, ct_ns_before(P, S), MAXB, INV, ct_swz2_out<N, S - 1>(), ct_swz2_out<N, S>()>(
        buf, nrows, rowstride, tw + d.tw_off[S], tid, nthr);
    fft_ct_stage_range<N, S + 1, E, MAXB, INV>(buf, nrows, rowstride, d, tw, tid, nthr);
  }
}

template <int N, int S, int MAXB, bool INV>
__device__ __forceinline__ void fft_ct_stages(float2* buf, int nrows, int rowstride, const FftDesc& d,
                                              const float2* __restrict__ tw, int tid, int nthr) {
  fft_ct_stage_range<N, S, ct_plan(N).ns, MAXB, INV>(buf, nrows, rowstride, d, tw, tid, nthr);
}

// fft_rows with a compile-time path for each length in SIZES (the generic
// path serves every other length).
template <bool ONE, bool INV, int... SIZES>
__device__ __forceinline__ void fft_rows_sized(float2* buf, int nrows, int rowstride, const FftDesc& d,
                                               const float2* __restrict__ tw, int tid, int nthr) {
  constexpr int MB = FftCfg<ONE>::MAXB;
  bool done = false;
  ((!done && d.n == SIZES ? (fft_ct_stages<SIZES, 0, MB, INV>(buf, nrows, rowstride, d, tw, tid, nthr),
                              done = true)
                          : false), ...);
  if (!done) fft_rows<ONE, INV>(buf, nrows, rowstride, d, tw, tid, nthr);
}

