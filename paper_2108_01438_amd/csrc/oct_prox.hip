// Proximal operators of Sec. 2.2-2.3 (eq. (12)-(14), (16)), FP64 reductions
// and small elementwise helpers.
//
// * l1 (Psi = I): complex soft threshold z = v max(0, 1 - tau/|v|).
// * Haar: a multi-level orthonormal Haar pyramid over the depth and lateral
//   axes is local to blocks of 2^levels samples per axis.  Each thread takes a
//   2x2(x2) group, keeps its soft-thresholded detail coefficients in registers
//   and hands the low band one level up through LDS; the coarsest low band is
//   left untouched and the synthesis walks back down.
// * TV: isotropic complex TV (forward differences, zero at the last index)
//   by the fast gradient projection (FGP) of Beck and Teboulle on the dual,
//   x = v + tau div p.  The 2-D path runs all inner steps of a tile in LDS
//   (temporal blocking with a halo as wide as the dependence cone); the
//   general path (volumes) runs one pass per inner step in global memory.
// All partial sums are per block in FP64 and summed in a fixed order.
#include "oct_fft.h"

namespace {

__device__ double block_sum(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) sh[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) s += sh[i];
  }
  return s;
}

__global__ void reduce_kernel(const double* __restrict__ p, int n, double* out, double scale, int accumulate) {
  __shared__ double sh[16];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) acc += p[i];
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) out[0] = accumulate ? out[0] + scale * s : scale * s;
}

__global__ void objective_kernel(const double* __restrict__ rp, int nr, const double* __restrict__ pp, int np,
                                 double lambda, double* out) {
  __shared__ double sh[16];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < nr; i += blockDim.x) a += rp[i];
  const double sa = block_sum(a, sh);
  __syncthreads();
  for (int i = threadIdx.x; i < np; i += blockDim.x) b += pp[i];
  const double sb = block_sum(b, sh);
  if (threadIdx.x == 0) out[0] = 0.5 * sa + lambda * sb;
}

__global__ void norm2_kernel(const float2* __restrict__ x, int64_t n, double* partial) {
  __shared__ double sh[16];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float2 v = x[i];
    acc += (double)v.x * v.x + (double)v.y * v.y;
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void scale_inv_sqrt_kernel(const float2* __restrict__ x, float2* y, int64_t n, const double* sumsq) {
  // a zero vector stays zero (the power iteration on Phi = 0 gives L = 0)
  const double ss = sumsq[0];
  const float sc = ss > 0.0 ? (float)(1.0 / sqrt(ss)) : 0.f;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = cscale(x[i], sc);
}

// SplitMix64 (Steele, Lea and Flood 2014) as a counter generator.
__device__ __forceinline__ uint64_t splitmix64(uint64_t counter, uint64_t seed) {
  uint64_t z = seed + (counter + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ double counter_uniform(uint64_t c, uint64_t seed) {
  return (double)(splitmix64(c, seed) >> 11) * 0x1.0p-52 - 1.0;
}

__global__ void uniform_kernel(float2* x, int64_t n, uint64_t seed) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = make_float2((float)counter_uniform(2ull * i, seed), (float)counter_uniform(2ull * i + 1ull, seed));
}

__global__ void copy_kernel(const float2* __restrict__ x, float2* y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = x[i];
}

// y[b][i] = s_b x[b][i] for items of per_item elements (T = float or float2)
template <typename T>
__global__ void scale_items_kernel(const T* __restrict__ x, T* y, int64_t per_item, int64_t n, ItemScales sc) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float f = sc.s[i / per_item];
    if constexpr (sizeof(T) == sizeof(float)) y[i] = x[i] * f;
    else y[i] = cscale(x[i], f);
  }
}

__global__ void zero_kernel(float2* y, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = make_float2(0.f, 0.f);
}

// soft threshold by tau, then the modulus clipped to bound (the projection onto
// C; exact for l1 because the constrained problem stays radial per pixel)
__global__ void prox_l1_kernel(const float2* __restrict__ v, float2* z, int64_t n, float tau, float bound,
                               double* partial) {
  __shared__ double sh[16];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float2 a = v[i];
    const float mag = sqrtf(a.x * a.x + a.y * a.y);
    const float sc = mag > tau ? fminf(1.f - tau / mag, bound / mag) : 0.f;
    const float2 r = make_float2(a.x * sc, a.y * sc);
    acc += (double)sqrtf(r.x * r.x + r.y * r.y);
    z[i] = r;
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0 && partial) partial[blockIdx.x] = s;
}

// ---------------------------------------------------------------------------
// Haar pyramid on blocks of 2^LV per axis.  D = 2 (depth, x) or 3 (depth, x, y).
// A workgroup covers NBN blocks along depth; level-l groups are indexed
// (a, b, c) with a along depth fastest.
// ---------------------------------------------------------------------------
constexpr float RS2 = 0.70710678118654752440f;

// analysis of one group in place: index bits (depth, x, y), 0 = low
template <int D>
__device__ __forceinline__ void haar_fwd_group(float2* v) {
#pragma unroll
  for (int ax = 0; ax < D; ++ax) {
    const int bit = 1 << ax;
#pragma unroll
    for (int i = 0; i < (1 << D); ++i) {
      if (i & bit) continue;
      const float2 e = v[i], o = v[i | bit];
      v[i] = make_float2((e.x + o.x) * RS2, (e.y + o.y) * RS2);
      v[i | bit] = make_float2((e.x - o.x) * RS2, (e.y - o.y) * RS2);
    }
  }
}
template <int D>
__device__ __forceinline__ void haar_inv_group(float2* v) {
#pragma unroll
  for (int ax = D - 1; ax >= 0; --ax) {
    const int bit = 1 << ax;
#pragma unroll
    for (int i = 0; i < (1 << D); ++i) {
      if (i & bit) continue;
      const float2 lo = v[i], hi = v[i | bit];
      v[i] = make_float2((lo.x + hi.x) * RS2, (lo.y + hi.y) * RS2);
      v[i | bit] = make_float2((lo.x - hi.x) * RS2, (lo.y - hi.y) * RS2);
    }
  }
}

// soft threshold; with PART the modulus of the result joins the l1 partial sum
template <bool PART>
__device__ __forceinline__ float2 soft(float2 a, float tau, double& acc) {
  const float mag = sqrtf(a.x * a.x + a.y * a.y);
  const float sc = mag > tau ? 1.f - tau / mag : 0.f;
  const float2 r = make_float2(a.x * sc, a.y * sc);
  if (PART) acc += (double)sqrtf(r.x * r.x + r.y * r.y);
  return r;
}

// PART: also the per-block FP64 sums of |detail coefficients| (the penalty
// value), only when the caller asks for them
template <int D, int LV, int NBN, bool PART>
__global__ void __launch_bounds__(1024) haar_kernel(ProxGeom g, const float2* __restrict__ vin, float2* zout,
                                                    float tau, double* partial) {
  constexpr int NV = 1 << D;
  constexpr int BS = 1 << LV;                     // block side
  constexpr int GA0 = NBN * BS / 2;               // level-0 groups along depth
  constexpr int GB0 = BS / 2;                     // along x (and y)
  constexpr int GC0 = (D == 3) ? BS / 2 : 1;
  constexpr int NG0 = GA0 * GB0 * GC0;
  __shared__ float2 ll[2][NG0];
  __shared__ double sh[16];
  const int tid = threadIdx.x;
  const int Nz = g.Nz, Nx = g.Nx, Ny = g.Ny;
  // tile origin
  const int tz = Nz / (NBN * BS) + ((Nz % (NBN * BS)) ? 1 : 0);
  const int tx = Nx / BS;
  const int ty = (D == 3) ? Ny / BS : 1;
  int t = blockIdx.x;
  const int iz = t % tz; t /= tz;
  const int ix = t % tx; t /= tx;
  const int iy = t % ty; t /= ty;
  const int b = t;
  const int z0 = iz * NBN * BS, x0 = ix * BS, y0 = iy * BS;
  // a 2x2(x2) group at depth 2a, x 2bb, y 2c of the tile: its first element's
  // offset; the others lie 1 (depth), sx (x) and sy (y) further
  const int64_t sx = Nz, sy = (int64_t)Nx * Nz;
  auto group_off = [&](int a, int bb, int c) -> int64_t {
    return (((int64_t)b * Ny + y0 + 2 * c) * Nx + x0 + 2 * bb) * Nz + z0 + 2 * a;
  };
  auto elem_off = [&](int i) -> int64_t { return (i & 1) + ((i >> 1) & 1) * sx + ((i >> 2) & 1) * sy; };

  float2 det[LV][NV];
  double acc = 0.0;
  // level 0: load a 2x2(x2) group
  {
    if (tid < NG0) {
      const int a = tid % GA0, bb = (tid / GA0) % GB0, c = tid / (GA0 * GB0);
      float2 v[NV];
      const bool ok = z0 + 2 * a < Nz;
      const float2* __restrict__ src = vin + group_off(a, bb, c);
#pragma unroll
      for (int i = 0; i < NV; ++i) v[i] = ok ? src[elem_off(i)] : make_float2(0.f, 0.f);
      haar_fwd_group<D>(v);
#pragma unroll
      for (int i = 1; i < NV; ++i) det[0][i] = soft<PART>(v[i], tau, acc);
      ll[0][tid] = v[0];
    }
  }
  __syncthreads();
  // analysis up the pyramid
  int GA = GA0, GB = GB0, GC = GC0;
#pragma unroll
  for (int l = 1; l < LV; ++l) {
    const int nA = GA / 2, nB = GB / 2, nC = (D == 3) ? GC / 2 : 1;
    const int src = (l - 1) & 1, dstb = l & 1;
    if (tid < nA * nB * nC) {
      const int a = tid % nA, bb = (tid / nA) % nB, c = tid / (nA * nB);
      float2 v[NV];
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        const int aa = 2 * a + (i & 1), b2 = 2 * bb + ((i >> 1) & 1), c2 = (D == 3) ? 2 * c + ((i >> 2) & 1) : 0;
        v[i] = ll[src][(c2 * GB + b2) * GA + aa];
      }
      haar_fwd_group<D>(v);
#pragma unroll
      for (int i = 1; i < NV; ++i) det[l][i] = soft<PART>(v[i], tau, acc);
      det[l][0] = v[0];   // coarsest low band kept (only used at l = LV-1)
      ll[dstb][tid] = v[0];
    }
    GA = nA; GB = nB; GC = nC;
    __syncthreads();
  }
  // synthesis down the pyramid (the top level keeps its low band)
#pragma unroll
  for (int l = LV - 1; l >= 1; --l) {
    // groups at level l: count GA*GB*GC (current sizes); parents write into ll[(l-1)&1]
    const int dstb = (l - 1) & 1;
    const int srcb = l & 1;
    if (tid < GA * GB * GC) {
      const int a = tid % GA, bb = (tid / GA) % GB, c = tid / (GA * GB);
      float2 v[NV];
      v[0] = (l == LV - 1) ? det[l][0] : ll[srcb][tid];
#pragma unroll
      for (int i = 1; i < NV; ++i) v[i] = det[l][i];
      haar_inv_group<D>(v);
      const int pA = GA * 2, pB = GB * 2;
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        const int aa = 2 * a + (i & 1), b2 = 2 * bb + ((i >> 1) & 1), c2 = (D == 3) ? 2 * c + ((i >> 2) & 1) : 0;
        ll[dstb][(c2 * pB + b2) * pA + aa] = v[i];
      }
    }
    GA *= 2; GB *= 2; if (D == 3) GC *= 2;
    __syncthreads();
  }
  if (tid < NG0) {
    const int a = tid % GA0, bb = (tid / GA0) % GB0, c = tid / (GA0 * GB0);
    float2 v[NV];
    v[0] = ll[0][tid];
#pragma unroll
    for (int i = 1; i < NV; ++i) v[i] = det[0][i];
    haar_inv_group<D>(v);
    if (z0 + 2 * a < Nz) {
      float2* __restrict__ dst = zout + group_off(a, bb, c);
#pragma unroll
      for (int i = 0; i < NV; ++i) dst[elem_off(i)] = v[i];
    }
  }
  if (PART) {
    const double s = block_sum(acc, sh);
    if (tid == 0) partial[blockIdx.x] = s;
  }
}

template <int D, int LV> struct HaarCfg;
template <int LV> struct HaarCfg<2, LV> { static constexpr int NBN = (LV <= 3) ? (256 >> (2 * LV - 2)) / 1 * 1 : 1; };
template <int LV> struct HaarCfg<3, LV> { static constexpr int NBN = (LV <= 2) ? 8 : (LV == 3 ? 4 : 1); };

template <int D, int LV>
int haar_threads() {
  constexpr int BS = 1 << LV;
  constexpr int NBN = HaarCfg<D, LV>::NBN;
  return NBN * (BS / 2) * (BS / 2) * (D == 3 ? BS / 2 : 1);
}

template <int D, int LV>
int haar_blocks(const ProxGeom& g) {
  constexpr int BS = 1 << LV;
  constexpr int NBN = HaarCfg<D, LV>::NBN;
  const int tz = (g.Nz + NBN * BS - 1) / (NBN * BS);
  return tz * (g.Nx / BS) * ((D == 3) ? g.Ny / BS : 1) * g.B;
}

template <int D, int LV>
hipError_t haar_launch(const ProxGeom& g, const float2* v, float2* z, float tau, double* partial, hipStream_t s) {
  constexpr int NBN = HaarCfg<D, LV>::NBN;
  const int nt = haar_threads<D, LV>();
  const int nb = haar_blocks<D, LV>(g);
  if (partial)
    hipLaunchKernelGGL((haar_kernel<D, LV, NBN, true>), dim3(nb), dim3(nt < 64 ? 64 : nt), 0, s, g, v, z, tau, partial);
  else
    hipLaunchKernelGGL((haar_kernel<D, LV, NBN, false>), dim3(nb), dim3(nt < 64 ? 64 : nt), 0, s, g, v, z, tau,
                       partial);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// TV by FGP, one pass per inner step (any dimension).
// strides: depth 1, x Nz, y Nx*Nz.  p, r: [nd][n] complex.
// ---------------------------------------------------------------------------
struct TvIdx {
  int Nz, Nx, Ny, nd;
  int64_t n;
  bool fast;              // n < 2^32: coordinates by 32-bit magic divisions
  FastDiv fz, fx, fy;
};

__device__ __forceinline__ void tv_coords(const TvIdx& d, int64_t i, int& iz, int& ix, int& iy) {
  if (d.fast) {
    const uint32_t u = (uint32_t)i, q1 = fdiv(u, d.fz), q2 = fdiv(q1, d.fx);
    iz = (int)(u - q1 * (uint32_t)d.Nz);
    ix = (int)(q1 - q2 * (uint32_t)d.Nx);
    iy = (int)(q2 - fdiv(q2, d.fy) * (uint32_t)d.Ny);
    return;
  }
  iz = (int)(i % d.Nz);
  const int64_t r = i / d.Nz;
  ix = (int)(r % d.Nx);
  iy = (int)((r / d.Nx) % d.Ny);
}

__device__ __forceinline__ float2 tv_div_at(const TvIdx& d, const float2* __restrict__ p, int64_t i, int iz,
                                            int ix, int iy) {
  float2 acc = make_float2(0.f, 0.f);
  const int64_t sx = d.Nz, sy = (int64_t)d.Nx * d.Nz;
  // depth
  if (iz < d.Nz - 1) acc = cadd(acc, p[i]);
  if (iz > 0) acc = csub(acc, p[i - 1]);
  // x
  if (ix < d.Nx - 1) acc = cadd(acc, p[d.n + i]);
  if (ix > 0) acc = csub(acc, p[d.n + i - sx]);
  if (d.nd == 3) {
    if (iy < d.Ny - 1) acc = cadd(acc, p[2 * d.n + i]);
    if (iy > 0) acc = csub(acc, p[2 * d.n + i - sy]);
  }
  return acc;
}

// out = P_C(v + tau div r), P_C the modulus clip to bound (+inf: none)
__global__ void tv_div_kernel(TvIdx d, const float2* __restrict__ v, const float2* __restrict__ r, float tau,
                              float bound, float2* out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < d.n; i += (int64_t)gridDim.x * blockDim.x) {
    int iz, ix, iy;
    tv_coords(d, i, iz, ix, iy);
    const float2 dv = tv_div_at(d, r, i, iz, ix, iy);
    const float2 a = v[i];
    float2 x = make_float2(a.x + tau * dv.x, a.y + tau * dv.y);
    const float m2 = x.x * x.x + x.y * x.y;
    if (m2 > bound * bound) x = cscale(x, bound * rsqrtf(m2));
    out[i] = x;
  }
}

__global__ void tv_step_kernel(TvIdx d, const float2* __restrict__ dd, float2* r, float2* p, float step, float mom) {
  const int64_t sx = d.Nz, sy = (int64_t)d.Nx * d.Nz;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < d.n; i += (int64_t)gridDim.x * blockDim.x) {
    int iz, ix, iy;
    tv_coords(d, i, iz, ix, iy);
    const float2 c = dd[i];
    float2 gz = (iz < d.Nz - 1) ? csub(dd[i + 1], c) : make_float2(0.f, 0.f);
    float2 gx = (ix < d.Nx - 1) ? csub(dd[i + sx], c) : make_float2(0.f, 0.f);
    float2 gy = make_float2(0.f, 0.f);
    if (d.nd == 3 && iy < d.Ny - 1) gy = csub(dd[i + sy], c);
    float2 pz = r[i], px = r[d.n + i], py = make_float2(0.f, 0.f);
    pz = make_float2(pz.x + step * gz.x, pz.y + step * gz.y);
    px = make_float2(px.x + step * gx.x, px.y + step * gx.y);
    float m2 = pz.x * pz.x + pz.y * pz.y + px.x * px.x + px.y * px.y;
    if (d.nd == 3) {
      py = r[2 * d.n + i];
      py = make_float2(py.x + step * gy.x, py.y + step * gy.y);
      m2 += py.x * py.x + py.y * py.y;
    }
    const float sc = m2 > 1.f ? 1.f / sqrtf(m2) : 1.f;
    pz = cscale(pz, sc);
    px = cscale(px, sc);
    py = cscale(py, sc);
    const float2 oz = p[i], ox = p[d.n + i];
    r[i] = make_float2(pz.x + mom * (pz.x - oz.x), pz.y + mom * (pz.y - oz.y));
    r[d.n + i] = make_float2(px.x + mom * (px.x - ox.x), px.y + mom * (px.y - ox.y));
    p[i] = pz;
    p[d.n + i] = px;
    if (d.nd == 3) {
      const float2 oy = p[2 * d.n + i];
      r[2 * d.n + i] = make_float2(py.x + mom * (py.x - oy.x), py.y + mom * (py.y - oy.y));
      p[2 * d.n + i] = py;
    }
  }
}

__global__ void tv_value_kernel(TvIdx d, const float2* __restrict__ z, double* partial) {
  __shared__ double sh[16];
  const int64_t sx = d.Nz, sy = (int64_t)d.Nx * d.Nz;
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < d.n; i += (int64_t)gridDim.x * blockDim.x) {
    int iz, ix, iy;
    tv_coords(d, i, iz, ix, iy);
    const float2 c = z[i];
    float m2 = 0.f;
    if (iz < d.Nz - 1) { const float2 g = csub(z[i + 1], c); m2 += g.x * g.x + g.y * g.y; }
    if (ix < d.Nx - 1) { const float2 g = csub(z[i + sx], c); m2 += g.x * g.x + g.y * g.y; }
    if (d.nd == 3 && iy < d.Ny - 1) { const float2 g = csub(z[i + sy], c); m2 += g.x * g.x + g.y * g.y; }
    acc += (double)sqrtf(m2);
  }
  const double s = block_sum(acc, sh);
  if (threadIdx.x == 0 && partial) partial[blockIdx.x] = s;
}

// ---------------------------------------------------------------------------
// 2-D TV by FGP with every inner step of a tile on chip.  Lane = depth sample
// (64 per wave, coalesced), each thread owns a strip of TV_S lateral samples
// in registers, 16 waves side by side laterally: a 64 x (16 TV_S) loaded
// tile.  Depth neighbours move by lane shuffles, lateral neighbours inside a
// strip are registers and across strips go through LDS.  One inner step
// reaches one sample further in every direction, so with a halo of
// n_inner + 1 the dual is exact on the core grown by one sample, which is
// what z = v + tau div p and TV(z) on the core need.
// ---------------------------------------------------------------------------
constexpr int TV_S = 8;
constexpr int TV_WAVES = 16;

// Whole-wave lane shifts (DPP wave_shr:1 / wave_shl:1, zero filled at the
// wave edge): lane i receives lane i-1 (shr) or lane i+1 (shl).
__device__ __forceinline__ float lane_prev(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float lane_next(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x130, 0xf, 0xf, true));
}

// The dual is kept zero wherever its component has no forward edge (last
// index along that axis, and every sample outside the image).  The step of
// such a component is zero too, so it stays zero, and the divergence needs
// no boundary tests: (div p)_i = p_i - p_{i-1} along each axis.
// BOUND: the constrained FGP of Beck and Teboulle, the primal point projected
// onto C = {|x_i| <= bound} in every step and at the end.
template <bool BOUND>
__global__ void __launch_bounds__(1024) tv2d_tile_kernel(Tv2dArgs a) {
  // strip-edge exchange rows: wave w publishes its last column in xr[w + 1]
  // and its first in xd[w]; xr[0] and xd[TV_WAVES] stay zero, so every read
  // is unconditional
  __shared__ float2 xr[TV_WAVES + 1][64];
  __shared__ float2 xd[TV_WAVES + 1][64];
  __shared__ double sh[16];
  // the wave index is uniform: strip positions and lateral edge weights stay in
  // scalar registers
  const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // Consecutive blocks go to the eight XCDs in turn; tile numbers are dealt
  // so that each XCD runs a run of consecutive tiles (depth neighbours, whose
  // halos overlap, share its L2).  The grid is padded to a multiple of 8.
  const int per = gridDim.x >> 3;
  const int bid = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (bid >= a.ntiles) return;
  const int tz = bid % a.ntz;
  const int tl = (bid / a.ntz) % a.ntl;
  const int b = bid / (a.ntz * a.ntl);
  const int Nz = a.Nz, Nx = a.Nx, H = a.H;
  const int cz0 = tz * a.CZ, cl0 = tl * a.CL;
  const int n = cz0 - H + lane;
  const int l0 = cl0 - H + w * TV_S;
  const bool nin = (n >= 0 && n < Nz);
  const bool zedge = (n >= 0 && n < Nz - 1);
  const int64_t ib = (int64_t)b * Nx * Nz;
  const int64_t N = a.n_total;
  const float tau = a.tau, step = a.step, bound = a.bound;
  const float sz = zedge ? step : 0.f;
  auto proj = [&](float2 x) __attribute__((always_inline)) {
    if (!BOUND) return x;
    const float sc = fminf(1.f, bound * __builtin_amdgcn_rsqf(x.x * x.x + x.y * x.y));
    return cscale(x, sc);
  };
  if (w == 0) xr[0][lane] = make_float2(0.f, 0.f);
  if (w == TV_WAVES - 1) xd[TV_WAVES][lane] = make_float2(0.f, 0.f);

  // FGP state per pixel: the extrapolated dual r and the previous dual P,
  // kept pre-multiplied by the momentum of the step that consumes it, so that
  // r = (1 + mom_k) p_k - mom_k p_{k-1} is one fused multiply-add per
  // component (mom after the last step is 1: P ends as the plain dual).  P is
  // updated in place: each pixel reads its old P before writing the new one.
  float2 v[TV_S], Pz[TV_S], Pl[TV_S], rz[TV_S], rl[TV_S];
  float sl[TV_S];
  const float mom0 = a.mom[0];
#pragma unroll
  for (int s = 0; s < TV_S; ++s) {
    const int l = l0 + s;
    const bool in = nin && l >= 0 && l < Nx;
    const bool ledge = l >= 0 && l < Nx - 1;
    sl[s] = ledge ? step : 0.f;
    const int64_t idx = ib + (int64_t)l * Nz + n;
    v[s] = in ? a.v[idx] : make_float2(0.f, 0.f);
    rz[s] = (in && zedge && a.pin) ? a.pin[idx] : make_float2(0.f, 0.f);
    rl[s] = (in && ledge && a.pin) ? a.pin[N + idx] : make_float2(0.f, 0.f);
    Pz[s] = cscale(rz[s], mom0);
    Pl[s] = cscale(rl[s], mom0);
  }
  for (int k = 0; k < a.n_inner; ++k) {
    const float mom1 = 1.f + a.mom[k];
    const float mnext = a.mom[k + 1];
    xr[w + 1][lane] = rl[TV_S - 1];
    __syncthreads();
    float2 d[TV_S];
#pragma unroll
    for (int s = 0; s < TV_S; ++s) {
      const float2 lp = (s > 0) ? rl[s - 1] : xr[w][lane];
      const float dx = (rz[s].x - lane_prev(rz[s].x)) + (rl[s].x - lp.x);
      const float dy = (rz[s].y - lane_prev(rz[s].y)) + (rl[s].y - lp.y);
      d[s] = proj(make_float2(fmaf(tau, dx, v[s].x), fmaf(tau, dy, v[s].y)));
    }
    xd[w][lane] = d[0];
    __syncthreads();
#pragma unroll
    for (int s = 0; s < TV_S; ++s) {
      const float2 dl = (s < TV_S - 1) ? d[s + 1] : xd[w + 1][lane];
      const float2 qz = make_float2(fmaf(sz, lane_next(d[s].x) - d[s].x, rz[s].x),
                                    fmaf(sz, lane_next(d[s].y) - d[s].y, rz[s].y));
      const float2 ql = make_float2(fmaf(sl[s], dl.x - d[s].x, rl[s].x), fmaf(sl[s], dl.y - d[s].y, rl[s].y));
      const float m2 = qz.x * qz.x + qz.y * qz.y + ql.x * ql.x + ql.y * ql.y;
      // projection onto |p| <= 1: 1/sqrt(m2) when m2 > 1, else 1 (m2 = 0 included)
      const float sc = fminf(1.f, __builtin_amdgcn_rsqf(m2));
      const float ca = mom1 * sc, cb = mnext * sc;
      rz[s] = make_float2(fmaf(ca, qz.x, -Pz[s].x), fmaf(ca, qz.y, -Pz[s].y));
      rl[s] = make_float2(fmaf(ca, ql.x, -Pl[s].x), fmaf(ca, ql.y, -Pl[s].y));
      Pz[s] = cscale(qz, cb);
      Pl[s] = cscale(ql, cb);
    }
  }
  // z = v + tau div p  (P holds p after the last step)
  xr[w + 1][lane] = Pl[TV_S - 1];
  __syncthreads();
  float2 z[TV_S];
#pragma unroll
  for (int s = 0; s < TV_S; ++s) {
    const float2 lp = (s > 0) ? Pl[s - 1] : xr[w][lane];
    const float dx = (Pz[s].x - lane_prev(Pz[s].x)) + (Pl[s].x - lp.x);
    const float dy = (Pz[s].y - lane_prev(Pz[s].y)) + (Pl[s].y - lp.y);
    z[s] = proj(make_float2(fmaf(tau, dx, v[s].x), fmaf(tau, dy, v[s].y)));
  }
  const bool zcore = nin && n >= cz0 && n < cz0 + a.CZ;
  if (a.partial) {   // TV(z) on the core as well, when the caller asks for it
    xd[w][lane] = z[0];
    __syncthreads();
    double acc = 0.0;
#pragma unroll
    for (int s = 0; s < TV_S; ++s) {
      const int l = l0 + s;
      const float dnx = lane_next(z[s].x), dny = lane_next(z[s].y);
      const float2 zl = (s < TV_S - 1) ? z[s + 1] : xd[w + 1][lane];
      if (zcore && l >= cl0 && l < cl0 + a.CL && l < Nx) {
        float m2 = 0.f;
        if (zedge) m2 += (dnx - z[s].x) * (dnx - z[s].x) + (dny - z[s].y) * (dny - z[s].y);
        if (l < Nx - 1) m2 += (zl.x - z[s].x) * (zl.x - z[s].x) + (zl.y - z[s].y) * (zl.y - z[s].y);
        acc += (double)sqrtf(m2);
      }
    }
    const double sum = block_sum(acc, sh);
    if (threadIdx.x == 0) a.partial[bid] = sum;
  }
#pragma unroll
  for (int s = 0; s < TV_S; ++s) {
    const int l = l0 + s;
    if (zcore && l >= cl0 && l < cl0 + a.CL && l < Nx) {
      const int64_t idx = ib + (int64_t)l * Nz + n;
      a.z[idx] = z[s];
      a.pout[idx] = Pz[s];
      a.pout[N + idx] = Pl[s];
    }
  }
}

int grid_for(int64_t n, int nt) {
  int64_t b = (n + nt - 1) / nt;
  if (b > 2048) b = 2048;
  if (b < 1) b = 1;
  return (int)b;
}

}  // namespace

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_reduce_sum(const double* partial, int n, double* out, double scale, int accumulate,
                             hipStream_t s) {
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(1024), 0, s, partial, n, out, scale, accumulate);
  return hipGetLastError();
}

hipError_t launch_objective(const double* rp, int nr, const double* pp, int np, double lambda, double* out,
                            hipStream_t s) {
  hipLaunchKernelGGL(objective_kernel, dim3(1), dim3(1024), 0, s, rp, nr, pp, np, lambda, out);
  return hipGetLastError();
}

hipError_t launch_norm2_partial(const float2* x, int64_t n, double* partial, int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(norm2_kernel, dim3(nblocks), dim3(256), 0, s, x, n, partial);
  return hipGetLastError();
}

hipError_t launch_scale_by_inv_sqrt(const float2* x, float2* y, int64_t n, const double* sumsq, hipStream_t s) {
  hipLaunchKernelGGL(scale_inv_sqrt_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, x, y, n, sumsq);
  return hipGetLastError();
}

hipError_t launch_fill_counter_uniform(float2* x, int64_t n, uint64_t seed, hipStream_t s) {
  hipLaunchKernelGGL(uniform_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, x, n, seed);
  return hipGetLastError();
}

hipError_t launch_copy(const float2* x, float2* y, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(copy_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, x, y, n);
  return hipGetLastError();
}

hipError_t launch_scale_items(const float* x, float* y, int64_t per_item, int items, const ItemScales& sc,
                              hipStream_t s) {
  const int64_t n = per_item * items;
  hipLaunchKernelGGL(scale_items_kernel<float>, dim3(grid_for(n, 256)), dim3(256), 0, s, x, y, per_item, n, sc);
  return hipGetLastError();
}

hipError_t launch_scale_items(const float2* x, float2* y, int64_t per_item, int items, const ItemScales& sc,
                              hipStream_t s) {
  const int64_t n = per_item * items;
  hipLaunchKernelGGL(scale_items_kernel<float2>, dim3(grid_for(n, 256)), dim3(256), 0, s, x, y, per_item, n, sc);
  return hipGetLastError();
}

hipError_t launch_zero(float2* x, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(zero_kernel, dim3(grid_for(n, 256)), dim3(256), 0, s, x, n);
  return hipGetLastError();
}

hipError_t launch_prox_l1(const float2* v, float2* z, int64_t n, float tau, float bound, double* partial,
                          int nblocks, hipStream_t s) {
  hipLaunchKernelGGL(prox_l1_kernel, dim3(nblocks), dim3(256), 0, s, v, z, n, tau, bound, partial);
  return hipGetLastError();
}

int haar_partials(const ProxGeom& g, int levels) {
  if (g.lateral_dims == 1) {
    switch (levels) {
      case 1: return haar_blocks<2, 1>(g);
      case 2: return haar_blocks<2, 2>(g);
      case 3: return haar_blocks<2, 3>(g);
      case 4: return haar_blocks<2, 4>(g);
      case 5: return haar_blocks<2, 5>(g);
    }
  } else {
    switch (levels) {
      case 1: return haar_blocks<3, 1>(g);
      case 2: return haar_blocks<3, 2>(g);
      case 3: return haar_blocks<3, 3>(g);
      case 4: return haar_blocks<3, 4>(g);
    }
  }
  return -1;
}

hipError_t launch_prox_haar(const ProxGeom& g, int levels, const float2* v, float2* z, float tau, double* partial,
                            hipStream_t s) {
  if (g.lateral_dims == 1) {
    switch (levels) {
      case 1: return haar_launch<2, 1>(g, v, z, tau, partial, s);
      case 2: return haar_launch<2, 2>(g, v, z, tau, partial, s);
      case 3: return haar_launch<2, 3>(g, v, z, tau, partial, s);
      case 4: return haar_launch<2, 4>(g, v, z, tau, partial, s);
      case 5: return haar_launch<2, 5>(g, v, z, tau, partial, s);
    }
  } else {
    switch (levels) {
      case 1: return haar_launch<3, 1>(g, v, z, tau, partial, s);
      case 2: return haar_launch<3, 2>(g, v, z, tau, partial, s);
      case 3: return haar_launch<3, 3>(g, v, z, tau, partial, s);
      case 4: return haar_launch<3, 4>(g, v, z, tau, partial, s);
    }
  }
  return hipErrorInvalidValue;
}

size_t tv_work_elems(const ProxGeom& g) {
  const int nd = g.lateral_dims + 1;
  const int64_t n = (int64_t)g.B * g.Ny * g.Nx * g.Nz;
  return (size_t)n * (size_t)(1 + nd);     // d, r of the general path
}

static bool tv_tiled(const ProxGeom& g, int n_inner) {
  return g.lateral_dims == 1 && n_inner >= 1 && n_inner <= TV_MAX_TILED_INNER;
}

static void tv2d_tiles(const ProxGeom& g, int n_inner, int* CZ, int* CL, int* ntz, int* ntl) {
  const int H = n_inner + 1;
  *CZ = 64 - 2 * H;
  *CL = TV_WAVES * TV_S - 2 * H;
  *ntz = (g.Nz + *CZ - 1) / *CZ;
  *ntl = (g.Nx + *CL - 1) / *CL;
}

int tv_partials(const ProxGeom& g, int n_inner) {
  if (tv_tiled(g, n_inner)) {
    int CZ, CL, ntz, ntl;
    tv2d_tiles(g, n_inner, &CZ, &CL, &ntz, &ntl);
    return ntz * ntl * g.B;
  }
  const int64_t n = (int64_t)g.B * g.Ny * g.Nx * g.Nz;
  return grid_for(n, 256);
}

// p_in (nullable = zero) -> p_out; z = v + tau div p_out; partial (nullable:
// not computed) = TV(z).
hipError_t launch_prox_tv(const ProxGeom& g, int n_inner, const float* mom, const float2* v, float2* z,
                          const float2* p_in, float2* p_out, float tau, float bound, double* partial,
                          float2* work, hipStream_t s) {
  if (tv_tiled(g, n_inner)) {
    Tv2dArgs a{};
    a.Nz = g.Nz;
    a.Nx = g.Nx;
    a.H = n_inner + 1;
    a.n_inner = n_inner;
    tv2d_tiles(g, n_inner, &a.CZ, &a.CL, &a.ntz, &a.ntl);
    a.n_total = (int64_t)g.B * g.Nx * g.Nz;
    a.tau = tau;
    a.step = 1.0f / (8.0f * tau);
    a.bound = bound;
    for (int k = 0; k < n_inner; ++k) a.mom[k] = mom[k];
    a.mom[n_inner] = 1.f;   // the last step leaves the plain dual in the kernel's P
    a.v = v;
    a.z = z;
    a.pin = p_in;
    a.pout = p_out;
    a.partial = partial;
    a.ntiles = a.ntz * a.ntl * g.B;
    const int nb = (a.ntiles + 7) & ~7;
    if (bound < INFINITY) hipLaunchKernelGGL(tv2d_tile_kernel<true>, dim3(nb), dim3(TV_WAVES * 64), 0, s, a);
    else hipLaunchKernelGGL(tv2d_tile_kernel<false>, dim3(nb), dim3(TV_WAVES * 64), 0, s, a);
    return hipGetLastError();
  }
  TvIdx d;
  d.Nz = g.Nz;
  d.Nx = g.Nx;
  d.Ny = (g.lateral_dims == 2) ? g.Ny : 1;
  d.nd = g.lateral_dims + 1;
  d.n = (int64_t)g.B * g.Ny * g.Nx * g.Nz;
  d.fast = d.n < (int64_t(1) << 32);
  d.fz = make_fastdiv((uint32_t)d.Nz);
  d.fx = make_fastdiv((uint32_t)d.Nx);
  d.fy = make_fastdiv((uint32_t)d.Ny);
  // batch items are independent: the y index wraps per item only for volumes;
  // for B-scans Ny = 1 and the x index never crosses a batch boundary because
  // coordinates are taken modulo each axis length.
  const int64_t np = d.n * d.nd;
  float2* dd = work;
  float2* r = work + d.n;
  const int gb = grid_for(d.n, 256);
  if (p_in) {
    hipLaunchKernelGGL(copy_kernel, dim3(grid_for(np, 256)), dim3(256), 0, s, p_in, p_out, np);
  } else {
    hipLaunchKernelGGL(zero_kernel, dim3(grid_for(np, 256)), dim3(256), 0, s, p_out, np);
  }
  hipLaunchKernelGGL(copy_kernel, dim3(grid_for(np, 256)), dim3(256), 0, s, p_out, r, np);
  const float step = 1.0f / (4.0f * d.nd * tau);
  for (int k = 0; k < n_inner; ++k) {
    hipLaunchKernelGGL(tv_div_kernel, dim3(gb), dim3(256), 0, s, d, v, r, tau, bound, dd);
    hipLaunchKernelGGL(tv_step_kernel, dim3(gb), dim3(256), 0, s, d, dd, r, p_out, step, mom[k]);
  }
  hipLaunchKernelGGL(tv_div_kernel, dim3(gb), dim3(256), 0, s, d, v, p_out, tau, bound, z);
  if (partial) hipLaunchKernelGGL(tv_value_kernel, dim3(gb), dim3(256), 0, s, d, z, partial);
  return hipGetLastError();
}
