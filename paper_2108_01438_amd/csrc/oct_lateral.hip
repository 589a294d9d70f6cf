// Lateral passes of the ISAM operator (Sec. 2.1, eq. (4) and the inverse
// transform that follows the filter in eq. (6)-(7)).
//
// One workgroup owns a tile of T consecutive rows (depth samples or
// spectrometer pixels) of one lateral line.  It pulls the tile into LDS
// (T contiguous complex values per A-scan: coalesced reads), transforms every
// row along the lateral axis in LDS, applies the mode's elementwise work and
// writes the tile back.  The elementwise work fused here:
//   * the real part, mask and residual of eq. (2) and the adjoint's lateral
//     transform (normal-operator seam, with FP64 partial sums of r^2);
//   * the FISTA extrapolation x = z + mu (z - z_prev) and gradient step of
//     eq. (15), and for l1 the complex soft threshold of eq. (13) followed by
//     the next iteration's forward lateral transform.
#include "oct_fft.h"

namespace {

__device__ __forceinline__ bool mask_bit(const uint32_t* __restrict__ mask, int words, int lat, int m) {
  return (mask[(int64_t)lat * words + (m >> 5)] >> (m & 31)) & 1u;
}

// Deterministic block sum of one double per thread (valid in thread 0).
__device__ double block_sum_d(double v, double* sh) {
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

template <int MODE, bool R7>
__global__ void __launch_bounds__(1024) lat_kernel(LatArgs a) {
  extern __shared__ float2 lds[];
  __shared__ double red[16];
  const int tid = threadIdx.x, nthr = blockDim.x;
  int bid = blockIdx.x;
  const int G = gridDim.x;
  if ((G & 7) == 0) {  // consecutive tiles of a line on the same XCD (shared L2)
    const int per = G >> 3;
    bid = (bid & 7) * per + (bid >> 3);
  }
  const LineGeom lg = a.lg;
  const int line = bid / a.n_tiles;
  const int tile = bid - line * a.n_tiles;
  const int r0 = tile * a.T;
  const int nr = min(a.T, lg.rows - r0);
  const int64_t base = (int64_t)(line / lg.ocnt) * lg.sa + (int64_t)(line % lg.ocnt) * lg.sb + r0;
  const int L = lg.L, T = a.T, rs = a.rowstride;
  const int latb = (line % lg.lat_lines) * L;
  const int n = L * T;

  float2* twl = lds + T * rs;   // twiddle table after the tile
  stage_twiddles(twl, a.tw, a.fd, tid, nthr);
  // ---- load the tile: element (row t, lateral l) -> lds[t * rs + l]
  for (int idx = tid; idx < n; idx += nthr) {
    const int l = idx >> a.log2T;
    const int t = idx & (T - 1);
    float2 v = make_float2(0.f, 0.f);
    if (t < nr) {
      const int64_t off = base + (int64_t)l * lg.es + t;
      if (MODE == LAT_ADJ_MEAS) {
        float r = a.srcf[off];
        if (a.mask && !mask_bit(a.mask, a.mask_words, latb + l, r0 + t)) r = 0.f;
        v = make_float2(r, 0.f);
      } else if (MODE == LAT_FFT && a.z != nullptr) {
        const float2 z = a.z[off], zo = a.zo[off];
        v = make_float2(z.x + a.mu * (z.x - zo.x), z.y + a.mu * (z.y - zo.y));
      } else {
        v = a.src[off];
      }
    }
    lds[t * rs + l] = v;
  }
  __syncthreads();

  if (a.inverse) fft_rows<R7, true>(lds, T, rs, a.fd, twl, tid, nthr);
  else fft_rows<R7, false>(lds, T, rs, a.fd, twl, tid, nthr);

  if (MODE == LAT_FFT || MODE == LAT_ADJ_MEAS) {
    for (int idx = tid; idx < n; idx += nthr) {
      const int l = idx >> a.log2T, t = idx & (T - 1);
      if (t < nr) a.dst[base + (int64_t)l * lg.es + t] = cscale(lds[t * rs + l], a.scale);
    }
    return;
  }
  if (MODE == LAT_FWD_MEAS) {
    for (int idx = tid; idx < n; idx += nthr) {
      const int l = idx >> a.log2T, t = idx & (T - 1);
      if (t < nr) {
        float yv = lds[t * rs + l].x * a.scale;
        if (a.mask && !mask_bit(a.mask, a.mask_words, latb + l, r0 + t)) yv = 0.f;
        a.dstf[base + (int64_t)l * lg.es + t] = yv;
      }
    }
    return;
  }
  if (MODE == LAT_UPDATE) {
    for (int idx = tid; idx < n; idx += nthr) {
      const int l = idx >> a.log2T, t = idx & (T - 1);
      if (t < nr) {
        const int64_t off = base + (int64_t)l * lg.es + t;
        const float2 g = cscale(lds[t * rs + l], a.scale);
        const float2 z = a.z[off], zo = a.zo[off];
        const float xr = z.x + a.mu * (z.x - zo.x), xi = z.y + a.mu * (z.y - zo.y);
        a.dst[off] = make_float2(xr - a.delta * g.x, xi - a.delta * g.y);
      }
    }
    return;
  }
  if (MODE == LAT_NORMAL) {
    double acc = 0.0;
    for (int idx = tid; idx < n; idx += nthr) {
      const int l = idx >> a.log2T, t = idx & (T - 1);
      float r = 0.f;
      if (t < nr) {
        const int64_t off = base + (int64_t)l * lg.es + t;
        const bool on = !a.mask || mask_bit(a.mask, a.mask_words, latb + l, r0 + t);
        if (on) r = lds[t * rs + l].x * a.scale - (a.y ? a.y[off] : 0.f);
      }
      acc += (double)r * (double)r;
      lds[t * rs + l] = make_float2(r, 0.f);
    }
    __syncthreads();
    fft_rows<R7, false>(lds, T, rs, a.fd, twl, tid, nthr);
    for (int idx = tid; idx < n; idx += nthr) {
      const int l = idx >> a.log2T, t = idx & (T - 1);
      if (t < nr) a.dst[base + (int64_t)l * lg.es + t] = cscale(lds[t * rs + l], a.scale2);
    }
    const double s = block_sum_d(acc, red);
    if (tid == 0 && a.partial) a.partial[bid] = s;
    return;
  }
  if (MODE == LAT_UPDATE_L1) {
    double acc = 0.0;
    for (int idx = tid; idx < n; idx += nthr) {
      const int l = idx >> a.log2T, t = idx & (T - 1);
      float2 xn = make_float2(0.f, 0.f);
      if (t < nr) {
        const int64_t off = base + (int64_t)l * lg.es + t;
        const float2 g = cscale(lds[t * rs + l], a.scale);
        const float2 z = a.z[off], zo = a.zo[off];
        const float vr = z.x + a.mu * (z.x - zo.x) - a.delta * g.x;
        const float vi = z.y + a.mu * (z.y - zo.y) - a.delta * g.y;
        const float mag = sqrtf(vr * vr + vi * vi);
        const float sc = mag > a.tau ? 1.f - a.tau / mag : 0.f;
        const float2 zn = make_float2(vr * sc, vi * sc);
        acc += (double)sqrtf(zn.x * zn.x + zn.y * zn.y);
        a.zo[off] = zn;
        xn = make_float2(zn.x + a.mu_next * (zn.x - z.x), zn.y + a.mu_next * (zn.y - z.y));
      }
      lds[t * rs + l] = xn;
    }
    __syncthreads();
    fft_rows<R7, false>(lds, T, rs, a.fd, twl, tid, nthr);
    for (int idx = tid; idx < n; idx += nthr) {
      const int l = idx >> a.log2T, t = idx & (T - 1);
      if (t < nr) a.dst[base + (int64_t)l * lg.es + t] = lds[t * rs + l];
    }
    const double s = block_sum_d(acc, red);
    if (tid == 0 && a.partial) a.partial[bid] = s;
    return;
  }
}

}  // namespace

// Rows per tile and threads per block: the tile (T rows of L complex) stays
// within 64 KB of LDS and every FFT stage fits 2 butterflies per thread.
int lateral_pick_tile(const LineGeom& lg, const FftDesc& fd, int* nthr, int* rowstride) {
  const int rs = (lg.L % 2 == 0) ? lg.L + 1 : lg.L;  // odd stride spreads LDS banks
  const int mb = fft_maxb(fd);
  const int64_t budget = 65280 - 8 * (int64_t)fft_tw_entries(fd);   // tile + twiddles within 64 KB
  int T = 32;
  while (T > 1 && (int64_t)T * rs * 8 > budget) T >>= 1;
  while (T > 1 && T > lg.rows) T >>= 1;
  for (; T >= 1; T >>= 1) {
    const int64_t bf = (int64_t)T * lg.L / fd.min_radix;
    for (int nt = 256; nt <= 1024; nt <<= 1) {
      if (bf <= mb * nt && (int64_t)T * rs * 8 <= budget) {
        *nthr = nt;
        *rowstride = rs;
        return T;
      }
    }
  }
  return 0;
}

template <bool R7>
hipError_t launch_lateral_t(LatMode mode, const LatArgs& a, hipStream_t s) {
  const size_t lds = ((size_t)a.T * a.rowstride + fft_tw_entries(a.fd)) * sizeof(float2);
  const int grid = a.lg.n_lines * a.n_tiles;
  const int mb = FftCfg<R7>::MAXB;
  int nthr = 256;
  {
    const int64_t bf = (int64_t)a.T * a.lg.L / a.fd.min_radix;
    while (nthr < 1024 && bf > (int64_t)mb * nthr) nthr <<= 1;
    if (bf > (int64_t)mb * nthr) return hipErrorInvalidConfiguration;
  }
  switch (mode) {
    case LAT_FFT: hipLaunchKernelGGL((lat_kernel<LAT_FFT, R7>), dim3(grid), dim3(nthr), lds, s, a); break;
    case LAT_FWD_MEAS: hipLaunchKernelGGL((lat_kernel<LAT_FWD_MEAS, R7>), dim3(grid), dim3(nthr), lds, s, a); break;
    case LAT_ADJ_MEAS: hipLaunchKernelGGL((lat_kernel<LAT_ADJ_MEAS, R7>), dim3(grid), dim3(nthr), lds, s, a); break;
    case LAT_NORMAL: hipLaunchKernelGGL((lat_kernel<LAT_NORMAL, R7>), dim3(grid), dim3(nthr), lds, s, a); break;
    case LAT_UPDATE: hipLaunchKernelGGL((lat_kernel<LAT_UPDATE, R7>), dim3(grid), dim3(nthr), lds, s, a); break;
    case LAT_UPDATE_L1: hipLaunchKernelGGL((lat_kernel<LAT_UPDATE_L1, R7>), dim3(grid), dim3(nthr), lds, s, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_lateral(LatMode mode, const LatArgs& a, hipStream_t s) {
  return fft_has7(a.fd) ? launch_lateral_t<true>(mode, a, s) : launch_lateral_t<false>(mode, a, s);
}
