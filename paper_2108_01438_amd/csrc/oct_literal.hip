// Q and D of the paper's literal chain (Sec. 2.1, eq. (6)-(9)), per
// lateral-frequency column, for M_k = 2N.
//
// Forward: the N samples of K (the filtered spectrum at the even detector
// wavenumbers, from the NUFFT column kernel) -> u = their N-point inverse DFT
// -> Q: N zeros appended -> D: 2N-point DFT -> times e^{j Omega_m}.
// Adjoint: times e^{-j Omega_m} -> D^H (unnormalised inverse 2N-point DFT) ->
// Q^T (first N) -> the adjoint of the N-point inverse DFT (DFT / N).
// One workgroup per column; the column lives in LDS for both transforms.
//
// The 2N-point DFT of u padded with N zeros is done as N-point transforms:
// its even outputs are DFT_N(u) = the N input samples themselves (u is their
// inverse DFT / N), its odd outputs DFT_N(u_n e^{-i pi n / N}).  Likewise
// the first N outputs of the unnormalised inverse 2N-point DFT of b are
// IDFT_N(b_even)_n + e^{i pi n / N} IDFT_N(b_odd)_n, and the DFT / N of the
// first term returns b_even.  Two N-point transforms per direction instead of
// an N-point and a 2N-point one, and N samples of LDS instead of 2N.
#include "oct_fft.h"

namespace {

template <bool ONE, bool ADJ>
__global__ void __launch_bounds__(1024) literal_dq_kernel(const float2* __restrict__ in, float2* __restrict__ out,
                                                          const float2* __restrict__ om, int N, FftDesc fN,
                                                          const float2* __restrict__ twN, FftDesc fM,
                                                          const float2* __restrict__ twM) {
  extern __shared__ float2 buf[];
  const int tid = threadIdx.x, nthr = blockDim.x;
  const int64_t c = blockIdx.x;
  const int M = 2 * N;
  const float inv = 1.f / (float)N;
  if (!ADJ) {
    const float2* src = in + c * N;
    for (int n = tid; n < N; n += nthr) buf[n] = src[n];
    __syncthreads();
    fft_rows_sized<ONE, true, OCT_CT_K_SIZES>(buf, 1, N, fN, twN, tid, nthr);
    for (int n = tid; n < N; n += nthr) {   // u_n e^{-i pi n / N}
      float sn, cs;
      sincospif(-(float)n / (float)N, &sn, &cs);
      buf[n] = cscale(cmul(buf[n], make_float2(cs, sn)), inv);
    }
    __syncthreads();
    fft_rows_sized<ONE, false, OCT_CT_K_SIZES>(buf, 1, N, fN, twN, tid, nthr);
    float2* dst = out + c * M;
    for (int k = tid; k < N; k += nthr) {
      dst[2 * k] = cmul(src[k], om[2 * k]);
      dst[2 * k + 1] = cmul(buf[k], om[2 * k + 1]);
    }
  } else {
    const float2* src = in + c * M;
    for (int k = tid; k < N; k += nthr) buf[k] = cmul(src[2 * k + 1], cconj(om[2 * k + 1]));
    __syncthreads();
    fft_rows_sized<ONE, true, OCT_CT_K_SIZES>(buf, 1, N, fN, twN, tid, nthr);
    for (int n = tid; n < N; n += nthr) {   // e^{i pi n / N} / N
      float sn, cs;
      sincospif((float)n / (float)N, &sn, &cs);
      buf[n] = cscale(cmul(buf[n], make_float2(cs, sn)), inv);
    }
    __syncthreads();
    fft_rows_sized<ONE, false, OCT_CT_K_SIZES>(buf, 1, N, fN, twN, tid, nthr);
    float2* dst = out + c * N;
    for (int k = tid; k < N; k += nthr) {
      const float2 be = cmul(src[2 * k], cconj(om[2 * k]));
      dst[k] = make_float2(be.x + buf[k].x, be.y + buf[k].y);
    }
  }
}

}  // namespace

// Threads per workgroup and the butterfly variant for transforms of N and 2N
// points in one block; 0 when no block of at most 1024 threads fits them.
int literal_dq_threads(const FftDesc& fN, const FftDesc& fM, bool* one) {
  const int64_t bN = fN.n / fN.min_radix, bM = fM.n / fM.min_radix;
  for (int nt = 256; nt <= 1024; nt <<= 1)
    if (bN <= nt && bM <= nt) {
      *one = true;
      return nt;
    }
  for (int nt = 256; nt <= 1024; nt <<= 1)
    if (bN <= 2 * nt && bM <= 2 * nt) {
      *one = false;
      return nt;
    }
  return 0;
}

hipError_t launch_literal_dq(bool adjoint, const float2* in, float2* out, const float2* om, int N, int64_t cols,
                             const FftDesc& fN, const float2* twN, const FftDesc& fM, const float2* twM,
                             hipStream_t s) {
  bool one = true;
  const int nt = literal_dq_threads(fN, fM, &one);
  if (nt == 0) return hipErrorInvalidConfiguration;
  const size_t lds = (size_t)N * sizeof(float2);
  const dim3 g((unsigned)cols), b(nt);
  if (one) {
    if (adjoint) hipLaunchKernelGGL((literal_dq_kernel<true, true>), g, b, lds, s, in, out, om, N, fN, twN, fM, twM);
    else hipLaunchKernelGGL((literal_dq_kernel<true, false>), g, b, lds, s, in, out, om, N, fN, twN, fM, twM);
  } else {
    if (adjoint) hipLaunchKernelGGL((literal_dq_kernel<false, true>), g, b, lds, s, in, out, om, N, fN, twN, fM, twM);
    else hipLaunchKernelGGL((literal_dq_kernel<false, false>), g, b, lds, s, in, out, om, N, fN, twN, fM, twM);
  }
  return hipGetLastError();
}
