// Direct (non-iterative) reconstructions of Sec. 3.1 and the evaluation
// metric of eq. (17).
//
// * The axial ("IFFT") and dispersion-corrected reconstructions of Figure 1
//   run the adjoint column kernel on every A-scan as a lateral-frequency-zero
//   column (beta = 2k, no beam term, no lateral transforms); this file
//   provides the spectrum-to-complex conversion in front of it.
// * The interpolated-ISAM baseline fills each A-scan's unobserved spectral
//   samples by linear interpolation in k before the ISAM adjoint.
// * NCC of magnitudes (eq. (17)) in FP64, two passes (means, then centred
//   sums), deterministic block partials.
// * The conjugate analytic signal of each A-scan along k, the operator A of
//   the paper's backward operator (eq. (10)-(11)).
#include "oct_fft.h"

#include <mutex>

// Scratch of the allocation-free NCC (oct_ncc_noalloc): the block partials of
// the two passes (3 x NCC_NOALLOC_MAX_BLOCKS doubles) followed by the five
// FP64 sums.  One copy per GPU, alive until the process ends; host code
// reaches it only through the address hipGetSymbolAddress returns for the
// current device (ncc_noalloc_scratch below).
static __device__ __align__(256) double scratch[NCC_NOALLOC_SCRATCH_DOUBLES];

namespace {

__device__ __forceinline__ bool observed(const uint32_t* __restrict__ mask, int words, int64_t lat, int m) {
  return !mask || ((mask[lat * words + (m >> 5)] >> (m & 31)) & 1u);
}

// W[i] = (s_i y_i, 0) over [batch][lat][Mk]
__global__ void meas_to_complex_kernel(const float* __restrict__ y, const uint32_t* __restrict__ mask, int words,
                                       int Mk, int Nlat, int64_t n, float2* __restrict__ W) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
    const int64_t row = i / Mk;
    const int m = (int)(i - row * Mk);
    W[i] = make_float2(observed(mask, words, row % Nlat, m) ? y[i] : 0.f, 0.f);
  }
}

// One block per A-scan: for every spectral pixel the last observed pixel at
// or before it and the first at or after it (two-level scans over per-thread
// chunks of at most 32 pixels: Mk <= 8192), then linear interpolation between
// them; the nearest observed value outside the observed range; zero when
// nothing is observed.
constexpr int INTERP_MAX_MK = 8192;
__global__ void __launch_bounds__(256) interp_fill_kernel(const float* __restrict__ y,
                                                          const uint32_t* __restrict__ mask, int words,
                                                          int Mk, int Nlat, float* __restrict__ out) {
  __shared__ int lastc[256], firstc[256];
  __shared__ short ridx[INTERP_MAX_MK];   // first observed pixel at or after m (Mk if none)
  const int tid = threadIdx.x, nt = blockDim.x;
  const int64_t row = blockIdx.x;
  const int64_t lat = row % Nlat;
  const float* yr = y + row * Mk;
  float* orow = out + row * Mk;
  const int Q = (Mk + nt - 1) / nt;
  const int c0 = min(tid * Q, Mk), c1 = min(c0 + Q, Mk);
  int lastobs = -1, firstobs = Mk;
  for (int m = c0; m < c1; ++m)
    if (observed(mask, words, lat, m)) {
      lastobs = m;
      if (firstobs == Mk) firstobs = m;
    }
  lastc[tid] = lastobs;
  firstc[tid] = firstobs;
  __syncthreads();
  // inclusive max-scan of lastc (left to right) and min-scan of firstc (right to left)
  for (int off = 1; off < nt; off <<= 1) {
    const int a = tid >= off ? lastc[tid - off] : -1;
    const int b = tid + off < nt ? firstc[tid + off] : Mk;
    __syncthreads();
    lastc[tid] = max(lastc[tid], a);
    firstc[tid] = min(firstc[tid], b);
    __syncthreads();
  }
  int right = tid + 1 < nt ? firstc[tid + 1] : Mk;   // first observed after this chunk
  for (int m = c1 - 1; m >= c0; --m) {
    if (observed(mask, words, lat, m)) right = m;
    ridx[m] = (short)right;
  }
  int left = tid > 0 ? lastc[tid - 1] : -1;          // last observed before this chunk
  for (int m = c0; m < c1; ++m) {
    if (observed(mask, words, lat, m)) left = m;
    const int R = ridx[m];
    float v;
    if (left == m) v = yr[m];
    else if (left < 0 && R >= Mk) v = 0.f;
    else if (left < 0) v = yr[R];
    else if (R >= Mk) v = yr[left];
    else {
      const float yl = yr[left], yh = yr[R];
      v = fmaf((yh - yl) / (float)(R - left), (float)(m - left), yl);
    }
    orow[m] = v;
  }
}

__device__ double block_sum_direct(double v, double* sh) {
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
  __syncthreads();
  return s;
}

__device__ __forceinline__ double cabs_d(float2 v) {
  return sqrt((double)v.x * (double)v.x + (double)v.y * (double)v.y);
}

// pass 0: sum |x|, sum |z|; pass 1 (means in mean[0..1]): centred products
__global__ void __launch_bounds__(256) ncc_partial_kernel(const float2* __restrict__ x, const float2* __restrict__ z,
                                                          int64_t n, int pass, const double* __restrict__ mean,
                                                          double* __restrict__ partial) {
  __shared__ double sh[8];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  const double mx = pass ? mean[0] : 0.0, mz = pass ? mean[1] : 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride) {
    const double a = cabs_d(x[i]) - mx, b = cabs_d(z[i]) - mz;
    if (pass == 0) {
      s0 += a;
      s1 += b;
    } else {
      s0 += a * b;
      s1 += a * a;
      s2 += b * b;
    }
  }
  const int nb = gridDim.x;
  const double t0 = block_sum_direct(s0, sh), t1 = block_sum_direct(s1, sh), t2 = block_sum_direct(s2, sh);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = t0;
    partial[nb + blockIdx.x] = t1;
    partial[2 * nb + blockIdx.x] = t2;
  }
}

// out[k] = scale * sum_b partial[k * nb + b], k < 3, in block order
__global__ void __launch_bounds__(256) ncc_reduce_kernel(const double* __restrict__ partial, int nb, double scale,
                                                         double* __restrict__ out) {
  __shared__ double sh[8];
  for (int k = 0; k < 3; ++k) {
    double s = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) s += partial[k * nb + i];
    const double t = block_sum_direct(s, sh);
    if (threadIdx.x == 0) out[k] = scale * t;
  }
}

// r = sum_xz / (sqrt(sum_xx) sqrt(sum_zz)) from the five sums of
// launch_ncc_sums (means, then the centred sums); NaN when either image has
// constant magnitude.
__global__ void ncc_finish_kernel(const double* __restrict__ dsc, double* __restrict__ r) {
  if (threadIdx.x == 0) {
    const double sxz = dsc[2], sxx = dsc[3], szz = dsc[4];
    r[0] = (sxx > 0.0 && szz > 0.0) ? sxz / (sqrt(sxx) * sqrt(szz)) : __builtin_nan("");
  }
}

// One block per A-scan: W = conj(analytic signal of s . r) along k, the
// operator A(z) = Re z - j H(z) of the paper's backward operator.  The
// analytic signal is the discrete one: forward FFT, negative frequencies
// removed, positive ones (below the Nyquist bin) doubled, inverse FFT.
template <bool ONE>
__global__ void __launch_bounds__(1024) analytic_conj_kernel(const float* __restrict__ r,
                                                             const uint32_t* __restrict__ mask, int words, int Mk,
                                                             int Nlat, FftDesc fM, const float2* __restrict__ twM,
                                                             float2* __restrict__ W) {
  extern __shared__ float2 row[];
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int64_t a = blockIdx.x;
  const int64_t lat = a % Nlat;
  const float* ra = r + a * Mk;
  for (int m = tid; m < Mk; m += nthr) row[m] = make_float2(observed(mask, words, lat, m) ? ra[m] : 0.f, 0.f);
  __syncthreads();
  fft_rows_sized<ONE, false, OCT_CT_K_SIZES>(row, 1, Mk, fM, twM, tid, nthr);
  const int half = Mk / 2;
  const float inv = 1.f / (float)Mk;
  for (int k = tid; k < Mk; k += nthr) {
    float h;
    if (k == 0 || ((Mk & 1) == 0 && k == half)) h = 1.f;
    else if (k < (Mk + 1) / 2) h = 2.f;
    else h = 0.f;
    row[k] = cscale(row[k], h * inv);
  }
  __syncthreads();
  fft_rows_sized<ONE, true, OCT_CT_K_SIZES>(row, 1, Mk, fM, twM, tid, nthr);
  float2* wa = W + a * Mk;
  for (int m = tid; m < Mk; m += nthr) wa[m] = cconj(row[m]);
}

}  // namespace

hipError_t launch_analytic_conj(const float* r, const uint32_t* mask, int words, int Mk, int Nlat, int64_t rows,
                                const FftDesc& fM, const float2* twM, float2* W, hipStream_t s) {
  const int bf = Mk / fM.min_radix;
  const int mb = fft_maxb(fM);
  int nt = 256;
  while (nt < 1024 && bf > mb * nt) nt <<= 1;
  if (bf > mb * nt) return hipErrorInvalidConfiguration;
  const size_t lds = (size_t)Mk * sizeof(float2);
  if (fft_one(fM, 1, nt))
    hipLaunchKernelGGL((analytic_conj_kernel<true>), dim3((unsigned)rows), dim3(nt), lds, s, r, mask, words, Mk, Nlat,
                       fM, twM, W);
  else
    hipLaunchKernelGGL((analytic_conj_kernel<false>), dim3((unsigned)rows), dim3(nt), lds, s, r, mask, words, Mk,
                       Nlat, fM, twM, W);
  return hipGetLastError();
}

hipError_t launch_meas_to_complex(const float* y, const uint32_t* mask, int words, int Mk, int Nlat, int64_t n,
                                  float2* W, hipStream_t s) {
  int64_t nb = (n + 255) / 256;
  if (nb > 4096) nb = 4096;
  hipLaunchKernelGGL(meas_to_complex_kernel, dim3((int)nb), dim3(256), 0, s, y, mask, words, Mk, Nlat, n, W);
  return hipGetLastError();
}

hipError_t launch_interp_fill(const float* y, const uint32_t* mask, int words, int Mk, int Nlat, int64_t rows,
                              float* out, hipStream_t s) {
  hipLaunchKernelGGL(interp_fill_kernel, dim3((unsigned)rows), dim3(256), 0, s, y, mask, words, Mk, Nlat, out);
  return hipGetLastError();
}

int ncc_blocks(int64_t n, int cap) {
  int64_t nb = (n + 255) / 256;
  if (nb > 1024) nb = 1024;
  if (nb > cap / 3) nb = cap / 3;
  return nb < 1 ? 1 : (int)nb;
}

hipError_t launch_ncc_sums(const float2* x, const float2* z, int64_t n, double* partial, int nb, double* dsc,
                           hipStream_t s) {
  hipLaunchKernelGGL(ncc_partial_kernel, dim3(nb), dim3(256), 0, s, x, z, n, 0, (const double*)nullptr, partial);
  hipLaunchKernelGGL(ncc_reduce_kernel, dim3(1), dim3(256), 0, s, (const double*)partial, nb, 1.0 / (double)n, dsc);
  hipLaunchKernelGGL(ncc_partial_kernel, dim3(nb), dim3(256), 0, s, x, z, n, 1, (const double*)dsc, partial);
  hipLaunchKernelGGL(ncc_reduce_kernel, dim3(1), dim3(256), 0, s, (const double*)partial, nb, 1.0, dsc + 2);
  return hipGetLastError();
}

hipError_t launch_ncc_finish(const double* dsc, double* r, hipStream_t s) {
  hipLaunchKernelGGL(ncc_finish_kernel, dim3(1), dim3(64), 0, s, dsc, r);
  return hipGetLastError();
}

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and cached; no allocation.
hipError_t ncc_noalloc_scratch(double** out) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static double* ptrs[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!ptrs[dev]) {
    double* p = nullptr;
    e = hipGetSymbolAddress(reinterpret_cast<void**>(&p), HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    ptrs[dev] = p;
  }
  *out = ptrs[dev];
  return hipSuccess;
}
