// Internal declarations shared by the host plan and the kernels of liboct.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define OCT_MAX_STAGES 16
#define OCT_KB_DEG 7             // degree of each KB polynomial piece
#define OCT_MAX_J 8
// transform lengths with compile-time FFT code: oversampled grids (sigma = 2
// on 512 .. 4096 depth samples) and lateral lengths of the common scan sizes
#define OCT_CT_K_SIZES 1024, 2048, 4096, 8192
#define OCT_CT_LAT_SIZES 64, 128, 256, 512, 1000, 1024

// Division of a 32-bit unsigned by a runtime constant d >= 1 through a
// multiply-high (Granlund-Montgomery round-up method): with l = ceil(log2 d),
// m = floor(2^32 (2^l - d) / d) + 1, q = (t + ((x - t) >> 1)) >> (l - 1),
// t = mulhi(m, x), exact for every 32-bit x; d = 1 is flagged by s = -1.
struct FastDiv {
  uint32_t m;
  int s;
  uint32_t d;
};

inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  if (d <= 1) {
    f.m = 0;
    f.s = -1;
    return f;
  }
  int l = 0;
  while ((1ull << l) < d) ++l;
  f.m = (uint32_t)((((1ull << 32) * ((1ull << l) - d)) / d) + 1);
  f.s = l - 1;
  return f;
}

// Mixed-radix factorisation of one transform length for the LDS Stockham FFT.
struct FftDesc {
  int n;
  int nstages;
  int radix[OCT_MAX_STAGES];
  int ns[OCT_MAX_STAGES];        // product of the radices before each stage
  FastDiv div_nb[OCT_MAX_STAGES];  // by n / radix (butterflies per row)
  FastDiv div_ns[OCT_MAX_STAGES];  // by ns
  int min_radix;
  // Per-stage twiddle rows: stage s (radix R, sub-transform size Ns > 1) owns
  // Ns rows of fft_tw_pad(R) entries at tw_off[s]; row k holds
  // e^{-2 pi i r k / (Ns R)} for r = 1..R-1, zero-padded to an even count.
  int tw_off[OCT_MAX_STAGES];
  int tw_total;
};

// entries per twiddle row of a radix-R stage: R - 1 rounded up to even (16-byte rows)
__host__ __device__ constexpr int fft_tw_pad(int R) { return R & ~1; }

// butterflies per thread the kernels may use for a transform of this shape
inline int fft_maxb(const FftDesc&) { return 2; }
// the one-butterfly variant serves every launch whose threads cover a stage
// of the narrowest radix
inline bool fft_one(const FftDesc& d, int64_t rows, int nthr) {
  return rows * (d.n / d.min_radix) <= nthr;
}

// Lines of a lateral transform.  Element (line o, lateral index l, row i) of a
// [.. ][lateral][rows] array lives at base(o) + l * es + i, with
// base(o) = (o / ocnt) * sa + (o % ocnt) * sb (all in elements).
struct LineGeom {
  int L;             // transform length
  int rows;          // rows per lateral position (n_depth or n_k)
  int n_lines;
  int ocnt;
  int64_t sa, sb, es;
  int lat_lines;     // lines per batch item that carry a mask (x-lines of a volume)
};

// Operation applied by the lateral pass around its transform.
enum LatMode {
  LAT_FFT = 0,        // dst = scale * FFT_sign(src)  [src optionally z + mu (z - zo)]
  LAT_FWD_MEAS = 1,   // y = s . Re( scale * IFFT(src) )                 -> float dst
  LAT_ADJ_MEAS = 2,   // dst = scale * FFT( s . r )                      <- float src
  LAT_NORMAL = 3,     // dst = scale2 * FFT( s . (Re(scale * IFFT(src)) - y) ), sum r^2
  LAT_UPDATE = 4,     // v = x - delta * scale * IFFT(src), x = z + mu (z - zo)
  LAT_UPDATE_L1 = 5,  // as UPDATE, then z' = soft(v), x' = z' + mu' (z' - z),
                      // z' -> zo, dst = FFT(x')
  LAT_RESID = 6       // dstf = s . (Re(scale * IFFT(src)) - y), sum r^2 (the residual alone)
};

struct LatArgs {
  LineGeom lg;
  FftDesc fd;
  const float2* tw;      // per-stage twiddle rows of the lateral transform
  int T;                 // rows per tile (a power of two)
  int log2T;
  int n_tiles;
  int rowstride;         // LDS row stride (>= L)
  int inverse;           // transform sign (+ when 1)
  float scale, scale2;
  // operands (meaning depends on mode)
  const float2* src;
  const float* srcf;
  float2* dst;
  float* dstf;
  const float* y;
  const uint32_t* mask;  // [lat][mask_words] bits, NULL = all observed
  int mask_words;
  // Half-spectrum storage of the spectral operand (x lines of the modes
  // FWD_MEAS, ADJ_MEAS and NORMAL): only lateral indices l <= L/2 are stored,
  // with line stride sa_half (0: full rows, line stride lg.sa).  The rows are
  // spectra of real rows, so l > L/2 holds conj(row[L - l]).
  int64_t sa_half;
  // x lines only: line strides of the source and destination operands when
  // they differ from lg.sa (0: lg.sa) -- a volume's spectral buffer pads
  // its y rows while the images it is transformed from and to do not
  int64_t sa_in, sa_out;
  const float2* z;       // current iterate z^{k-1} (UPDATE: the extrapolated x itself when zo is NULL)
  float2* zo;            // previous iterate z^{k-2}; receives z^k in UPDATE_L1
  float2* xout;          // FFT with z: also stores x = z + mu (z - zo) here (nullable)
  float mu;              // momentum forming x from (z, zo)
  float mu_next;         // momentum forming the next x (UPDATE_L1)
  float delta;
  float tau;
  float bound;           // UPDATE_L1: modulus bound of the constraint set (+inf: none)
  double* partial;       // per-block FP64 partial sums (NORMAL: 1/2 r^2; UPDATE_L1: |z'|)
};

struct NufftArgs {
  int Nz, Mk, K, nc, J, Nlat;
  int n_cols;
  // image-side columns: lateral index y n_x + x of batch item b lives at
  // ((b n_y + y) xs + x) Nz (xs = n_x: dense; n_x + 1: a volume's padded
  // spectral buffer)
  int Nx, xs;
  double ct;             // K dz / (2 pi): oversampled-grid coordinate per unit beta
  double invK;           // 1 / K
  double df;             // z_f - n_c dz (focus offset); 0 skips its phase
  double k_min, dk;      // linear wavenumber grid k_m = k_min + m dk
  const double* k2x4;    // [Mk] 4 k_m^2
  const float2* phase;   // [Mk] e^{j(-2 k_m z_f + Omega_m)}
  const double* q2;      // [Nlat] |q|^2
  const float* beam;     // [Nlat] e^{-q^2 w0^2 / 8}
  const float* deap;     // [Nz] 1 / Psi0((n - n_c) / K)
  const float* kbc;      // [J/2][even, odd][(OCT_KB_DEG+1)/2] KB pieces in x = 2f - 1
  FftDesc fK;
  const float2* twK;     // per-stage twiddle rows of the K-point transform
  // Column pairs (q, -q) of the half-spectrum kernels: {column of q, column of
  // -q, half-spectrum slot of q, half-spectrum slot of -q or -1}, per batch
  // item; n_half = half-spectrum columns per batch item (n_y (n_x / 2 + 1)).
  const int4* pairs;
  int n_pairs;
  int n_half;
};

// Residual output of the forward pair kernel (every pixel observed): R^ =
// W_h / N_lat - yh, and per-block N_lat-weighted |R^|^2 into partial (NULL:
// none); yh NULL stands for y = 0.
struct PairRes {
  const float2* yh;
  double* partial;
  float inv_nlat;
  double nlat;
};

// Launchers (kernels in the .hip files; all asynchronous on `s`).
hipError_t launch_lateral(LatMode mode, const LatArgs& a, hipStream_t s);
int lateral_pick_tile(const LineGeom& lg, const FftDesc& fd, int* nthr, int* rowstride);
hipError_t launch_nufft_fwd(const NufftArgs& a, const float2* X1, float2* W, hipStream_t s);
hipError_t launch_nufft_adj(const NufftArgs& a, const float2* Rh, float2* X, hipStream_t s);
size_t nufft_adj_lds_bytes(const NufftArgs& a);
// Half-spectrum column kernels: W_h(q) = (W(q) + conj W(-q)) / 2 from the
// columns q and -q of X1, and both image columns from R^(q) (R^(-q) = conj R^(q)).
hipError_t launch_nufft_fwd_pair(const NufftArgs& a, const float2* X1, float2* Wh, hipStream_t s);
hipError_t launch_nufft_adj_pair(const NufftArgs& a, const float2* Rh, float2* X, hipStream_t s);
// The forward pair kernel with the residual seam of a fully observed plan:
// Rh = W_h / N_lat - yh (yh may be Rh itself, or NULL for y = 0), the
// residual norm partials (one per block, n_pairs * batch) into partial when
// that is not NULL.
hipError_t launch_nufft_fwd_pair_res(const NufftArgs& a, const float2* X1, float2* Rh, const float2* yh,
                                     double* partial, hipStream_t s);
size_t nufft_pair_lds_bytes(const NufftArgs& a, bool adjoint);
// Fully observed plans: both column kernels of a pair in one launch, X1 ->
// R^ = W_h / N_lat - yh (kept in registers; residual partials as above) ->
// X = the adjoint columns (X may be X1: a pair reads its columns before it
// writes them).  Supported when every thread's samples fit its registers.
hipError_t launch_nufft_normal_pair(const NufftArgs& a, const float2* X1, const float2* yh, double* partial,
                                    float2* X, hipStream_t s);
size_t nufft_normal_pair_lds_bytes(const NufftArgs& a);
bool nufft_normal_pair_supported(const NufftArgs& a);
bool nufft_pair_supported(const NufftArgs& a);   // LDS and thread limits of the pair kernels

// Reductions and elementwise helpers.
hipError_t launch_reduce_sum(const double* partial, int n, double* out, double scale,
                             int accumulate, hipStream_t s);
hipError_t launch_norm2_partial(const float2* x, int64_t n, double* partial, int nblocks,
                                hipStream_t s);
hipError_t launch_scale_by_inv_sqrt(const float2* x, float2* y, int64_t n, const double* sumsq,
                                    hipStream_t s);
hipError_t launch_fill_counter_uniform(float2* x, int64_t n, uint64_t seed, hipStream_t s);
hipError_t launch_copy(const float2* x, float2* y, int64_t n, hipStream_t s);
// per-item scale factors passed by value (no device copy): at most OCT_MAX_LAMBDA_ITEMS items
struct ItemScales {
  float s[64];
};
hipError_t launch_scale_items(const float* x, float* y, int64_t per_item, int items, const ItemScales& sc,
                              hipStream_t s);
hipError_t launch_scale_items(const float2* x, float2* y, int64_t per_item, int items, const ItemScales& sc,
                              hipStream_t s);
hipError_t launch_zero(float2* x, int64_t n, hipStream_t s);
hipError_t launch_objective(const double* res_partial, int nres, const double* pen_partial,
                            int npen, double lambda, double* out, hipStream_t s);

// Conjugate analytic signal of each A-scan's spectrum (Hilbert transform along k).
hipError_t launch_analytic_conj(const float* r, const uint32_t* mask, int words, int Mk, int Nlat, int64_t rows,
                                const FftDesc& fM, const float2* twM, float2* W, hipStream_t s);

// Q and D of the literal chain (M_k = 2N) per lateral-frequency column: forward
// N samples of K -> 2N spectra with e^{j Omega}; adjoint the reverse.
int literal_dq_threads(const FftDesc& fN, const FftDesc& fM, bool* one);
hipError_t launch_literal_dq(bool adjoint, const float2* in, float2* out, const float2* om, int N, int64_t cols,
                             const FftDesc& fN, const float2* twN, const FftDesc& fM, const float2* twM,
                             hipStream_t s);

// Direct reconstructions and the NCC metric.
hipError_t launch_meas_to_complex(const float* y, const uint32_t* mask, int words, int Mk, int Nlat, int64_t n,
                                  float2* W, hipStream_t s);
hipError_t launch_interp_fill(const float* y, const uint32_t* mask, int words, int Mk, int Nlat, int64_t rows,
                              float* out, hipStream_t s);
int ncc_blocks(int64_t n, int cap);
// allocation-free NCC: block partials of at most NCC_NOALLOC_MAX_BLOCKS blocks
// (the count oct_ncc uses for any n) and the five sums, in a static device array
constexpr int NCC_NOALLOC_MAX_BLOCKS = 1024;
constexpr int NCC_NOALLOC_SCRATCH_DOUBLES = 3 * NCC_NOALLOC_MAX_BLOCKS + 8;
hipError_t ncc_noalloc_scratch(double** out);
hipError_t launch_ncc_finish(const double* dsc, double* r, hipStream_t s);
// means -> dsc[0..1], centred sums (xz, xx, zz) -> dsc[2..4]; partial holds 3 * nb doubles
hipError_t launch_ncc_sums(const float2* x, const float2* z, int64_t n, double* partial, int nb, double* dsc,
                           hipStream_t s);

// Proximal operators.
struct ProxGeom {
  int B, Ny, Nx, Nz;     // image [B][Ny][Nx][Nz]
  int lateral_dims;
};
// bound: modulus bound of the constraint set C of eq. (16), +inf for C = C^N
hipError_t launch_prox_l1(const float2* v, float2* z, int64_t n, float tau, float bound, double* partial,
                          int nblocks, hipStream_t s);
int haar_partials(const ProxGeom& g, int levels);
hipError_t launch_prox_haar(const ProxGeom& g, int levels, const float2* v, float2* z,
                            float tau, double* partial, hipStream_t s);
int tv_partials(const ProxGeom& g, int n_inner);
hipError_t launch_prox_tv(const ProxGeom& g, int n_inner, const float* mom, const float2* v,
                          float2* z, const float2* p_in, float2* p_out, float tau, float bound,
                          double* partial, float2* work, hipStream_t s);
size_t tv_work_elems(const ProxGeom& g);
// DT-CWT: z = W^T soft_tau(W v); work holds dtcwt_work_elems complex values
// (B-scan: four trees and four staging arrays; volume: eight trees and sixteen
// staging arrays); the value pass writes sum |W x| over the detail bands as
// dtcwt_partials block partials.
int dtcwt_partials(const ProxGeom& g, int levels);
size_t dtcwt_work_elems(const ProxGeom& g);
hipError_t launch_prox_dtcwt(const ProxGeom& g, int levels, const float2* v, float2* z, float tau,
                             float2* work, hipStream_t s);
hipError_t launch_dtcwt_value(const ProxGeom& g, int levels, const float2* x, float2* work,
                              double* partial, hipStream_t s);
void dtcwt_filter_taps(int which, float* h0, int* n);

// 2-D TV tile kernel arguments (inner steps up to TV_MAX_TILED_INNER).
#define TV_MAX_TILED_INNER 27
struct Tv2dArgs {
  int Nz, Nx, H, n_inner, CZ, CL, ntz, ntl;
  int ntiles;               // ntz * ntl * batch (the launch is padded to a multiple of 8)
  int64_t n_total;          // image elements (stride between dual components)
  float tau, step;
  float bound;              // modulus bound of the constraint set (used when the kernel is built for it)
  float mom[TV_MAX_TILED_INNER + 1];
  const float2* v;
  float2* z;
  const float2* pin;        // nullable: cold start
  float2* pout;
  double* partial;
};
