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

// Real-part pairing.  Only Re ifft(W) of a spectrum row W is ever used, and
// Re ifft(W) = ifft(W_h) with the Hermitian part W_h(q) = (W(q) + conj W(-q)) / 2.
// Row p (p < H = T/2) is replaced by W_h[p] + j W_h[p + H], so one complex
// inverse transform yields the real parts of two rows (in .x and .y).
__device__ __forceinline__ void pack_real_pairs(float2* lds, int H, int rs, int L, int tid, int nthr) {
  const int hl = L / 2 + 1;
  for (int p = 0; p < H; ++p) {
    float2* ra = lds + p * rs;
    const float2* rb = lds + (p + H) * rs;
    for (int q = tid; q < hl; q += nthr) {
      const int mq = q == 0 ? 0 : L - q;
      const float2 a0 = ra[q], a1 = ra[mq], b0 = rb[q], b1 = rb[mq];
      const float2 ha = make_float2(0.5f * (a0.x + a1.x), 0.5f * (a0.y - a1.y));   // W_h[p](q)
      const float2 hb = make_float2(0.5f * (b0.x + b1.x), 0.5f * (b0.y - b1.y));   // W_h[p+H](q)
      ra[q] = make_float2(ha.x - hb.y, ha.y + hb.x);
      ra[mq] = make_float2(ha.x + hb.y, hb.x - ha.y);   // conj ha + j conj hb
    }
  }
}

// After a forward transform of rows holding r_p + j r_{p+H} (both real), the
// spectrum of tile row t: Z = fft(row t mod H), R_p = (Z(q) + conj Z(-q)) / 2,
// R_{p+H} = (Z(q) - conj Z(-q)) / 2j.
__device__ __forceinline__ float2 unpack_real_pair(const float2* lds, int rs, int L, int H, int t, int l) {
  const bool second = t >= H;
  const float2* row = lds + (second ? t - H : t) * rs;
  const float2 z0 = row[l], z1 = row[l == 0 ? 0 : L - l];
  return second ? make_float2(0.5f * (z0.y + z1.y), 0.5f * (z1.x - z0.x))
                : make_float2(0.5f * (z0.x + z1.x), 0.5f * (z0.y - z1.y));
}

struct Z2 {
  float2 a, b;
};
struct FM {
  float f;
  uint32_t m;
};
struct YM {
  float ya, yb;
  uint32_t ma, mb;
};

// float2 slots of the tile in LDS, rounded up to keep the twiddle rows that
// follow it 16-byte aligned
__host__ __device__ inline int lat_tile_f2(int T, int rs) { return (T * rs + 1) & ~1; }

template <int MODE, bool ONE>
__global__ void __launch_bounds__(1024) lat_kernel(LatArgs a) {
  extern __shared__ float2 lds[];
  __shared__ double red[16];
  const int tid = threadIdx.x, nthr = blockDim.x;
  // Consecutive blocks go to the eight XCDs in turn; tile numbers are dealt
  // so that each XCD runs consecutive tiles of a line (their rows share cache
  // lines in its L2).  The grid is padded to a multiple of 8.
  const int per = gridDim.x >> 3;
  const int bid = (int)(blockIdx.x & 7) * per + (int)(blockIdx.x >> 3);
  if (bid >= a.lg.n_lines * a.n_tiles) return;
  const LineGeom lg = a.lg;
  const int line = bid / a.n_tiles;
  const int tile = bid - line * a.n_tiles;
  const int r0 = tile * a.T;
  const int nr = min(a.T, lg.rows - r0);
  const int64_t base = (int64_t)(line / lg.ocnt) * lg.sa + (int64_t)(line % lg.ocnt) * lg.sb + r0;
  const int L = lg.L, T = a.T, rs = a.rowstride;
  // spectral operand in half-spectrum storage (x lines only: ocnt = 1, sb = 0)
  const bool half = a.sa_half != 0;
  const int Lh = L / 2 + 1;
  const int64_t hbase = half ? (int64_t)line * a.sa_half + r0 : base;
  const int latb = (line % lg.lat_lines) * L;
  const int n = L * T;
  const int lt = a.log2T;

  // The transform's twiddle rows are copied next to the tile, so the
  // transform waits on no global load (the late loads below stay in flight
  // through it).
  float2* twl = lds + lat_tile_f2(T, rs);
  {
    const float4* __restrict__ s4 = reinterpret_cast<const float4*>(a.tw);
    float4* d4 = reinterpret_cast<float4*>(twl);
    for (int i = tid; i < (a.fd.tw_total >> 1); i += nthr) d4[i] = s4[i];
  }
  // modes that need only real parts (or transform real rows) pair rows p and p + H
  constexpr bool REAL_PAIRS = MODE == LAT_FWD_MEAS || MODE == LAT_ADJ_MEAS || MODE == LAT_NORMAL ||
                               MODE == LAT_RESID;
  const bool pair = REAL_PAIRS && T >= 2;
  const int H = T >> 1;
  const int nrow_t = pair ? H : T;   // rows that go through the transforms
  // global offset of tile element idx (row t = idx mod T, lateral l = idx / T); rows past the
  // image (ragged last tile) are clamped to a valid row and masked by the caller
  auto goff = [&](int idx) -> int64_t {
    const int l = idx >> lt, t = min(idx & (T - 1), nr - 1);
    return base + (int64_t)l * lg.es + t;
  };
  auto mword = [&](int l, int row) -> uint32_t {
    return a.mask ? a.mask[(int64_t)(latb + l) * a.mask_words + (row >> 5)] : ~0u;
  };

  // Loads consumed after the transform (the extrapolated point, or the
  // iterate pair z, z_prev it comes from, of the gradient step; the data and
  // mask of the normal seam).  When they fit
  // PF per thread they are issued right after the tile's own loads and stream
  // in while the tile is transformed (load counters retire in order, so they
  // must come after every load the transform waits for).
  constexpr bool LATE_Z = MODE == LAT_UPDATE || MODE == LAT_UPDATE_L1;
  constexpr bool LATE_Y = MODE == LAT_NORMAL;
  constexpr int PF = 8;
  const int log2H = lt - 1;
  auto load_z = [&](int idx) {
    const int64_t o = goff(idx);
    return Z2{a.z[o], a.zo ? a.zo[o] : make_float2(0.f, 0.f)};
  };
  auto load_y = [&](int idx) {
    const int l = idx >> log2H, p = idx & (H - 1);
    const int pa = min(p, nr - 1), pb = min(p + H, nr - 1);
    const int64_t oa = base + (int64_t)l * lg.es + pa, ob = base + (int64_t)l * lg.es + pb;
    return YM{a.y ? a.y[oa] : 0.f, a.y ? a.y[ob] : 0.f, mword(l, r0 + pa), mword(l, r0 + pb)};
  };
  using Late = std::conditional_t<LATE_Y, YM, Z2>;
  const int n_late = LATE_Y ? (n >> 1) : n;
  const bool early = (LATE_Z || (LATE_Y && pair)) && n_late <= PF * nthr;
  Late pf[PF];
  // run use(idx, value) over the late elements, prefetched or loaded now
  auto late_for = [&](auto load, auto use) __attribute__((always_inline)) {
    if (early) {
#pragma unroll
      for (int i = 0; i < PF; ++i) {
        const int idx = tid + i * nthr;
        if (idx < n_late) use(idx, pf[i]);
      }
    } else {
      batched_for(n_late, tid, nthr, load, use);
    }
  };

  // ---- load the tile: element (row t, lateral l) -> lds[t * rs + l]
  if (MODE == LAT_ADJ_MEAS) {
    // real rows; paired: row t -> component t >= H of row t mod H
    float* ldsf = reinterpret_cast<float*>(lds);
    batched_for(n, tid, nthr,
      [&](int idx) { const int l = idx >> lt, t = min(idx & (T - 1), nr - 1);
                     return FM{a.srcf[goff(idx)], mword(l, r0 + t)}; },
      [&](int idx, FM v) {
        const int l = idx >> lt, t = idx & (T - 1);
        const float r = (t < nr && ((v.m >> ((r0 + t) & 31)) & 1u)) ? v.f : 0.f;
        if (pair) ldsf[2 * ((t < H ? t : t - H) * rs + l) + (t < H ? 0 : 1)] = r;
        else lds[t * rs + l] = make_float2(r, 0.f);
      });
  } else if (MODE == LAT_FFT && a.z != nullptr) {
    batched_for(n, tid, nthr,
      [&](int idx) { const int64_t o = goff(idx); return Z2{a.z[o], a.zo[o]}; },
      [&](int idx, Z2 v) {
        const int l = idx >> lt, t = idx & (T - 1);
        float2 x;
        {
          // x = z + mu (z - z_prev) rounded step by step, as the fused l1 update
          // forms it: a resumed solve then matches an uninterrupted one bitwise
#pragma clang fp contract(off)
          x = make_float2(v.a.x + a.mu * (v.a.x - v.b.x), v.a.y + a.mu * (v.a.y - v.b.y));
        }
        lds[t * rs + l] = t < nr ? x : make_float2(0.f, 0.f);
        if (a.xout && t < nr) a.xout[base + (int64_t)l * lg.es + t] = x;
      });
  } else if ((MODE == LAT_FWD_MEAS || MODE == LAT_NORMAL) && half) {
    // half rows of Hermitian spectra, extended: row[L - l] = conj(row[l]); at
    // l = 0 (and L/2) only the real part belongs to the Hermitian row.
    // Paired: row p <- row_p + j row_{p+H}, so that one inverse transform
    // gives the real rows p and p + H (in .x and .y).
    auto hoff = [&](int l, int t) -> int64_t { return hbase + (int64_t)l * lg.es + min(t, nr - 1); };
    if (pair) {
      const int log2H = lt - 1;
      batched_for(Lh * H, tid, nthr,
        [&](int idx) { const int l = idx >> log2H, p = idx & (H - 1);
                       return Z2{a.src[hoff(l, p)], a.src[hoff(l, p + H)]}; },
        [&](int idx, Z2 v) {
          const int l = idx >> log2H, p = idx & (H - 1);
          float2 va = p < nr ? v.a : make_float2(0.f, 0.f), vb = p + H < nr ? v.b : make_float2(0.f, 0.f);
          const bool self = l == 0 || 2 * l == L;
          if (self) { va.y = 0.f; vb.y = 0.f; }
          float2* ra = lds + p * rs;
          ra[l] = make_float2(va.x - vb.y, va.y + vb.x);
          if (!self) ra[L - l] = make_float2(va.x + vb.y, vb.x - va.y);
        });
    } else {
      batched_for(Lh * T, tid, nthr,
        [&](int idx) { return a.src[hoff(idx >> lt, idx & (T - 1))]; },
        [&](int idx, float2 v) {
          const int l = idx >> lt, t = idx & (T - 1);
          if (t >= nr) v = make_float2(0.f, 0.f);
          const bool self = l == 0 || 2 * l == L;
          if (self) v.y = 0.f;
          lds[t * rs + l] = v;
          if (!self) lds[t * rs + L - l] = cconj(v);
        });
    }
  } else {
    batched_for(n, tid, nthr,
      [&](int idx) { return a.src[goff(idx)]; },
      [&](int idx, float2 v) {
        const int l = idx >> lt, t = idx & (T - 1);
        lds[t * rs + l] = t < nr ? v : make_float2(0.f, 0.f);
      });
  }
  // retire the tile's loads (including the clamped ones nobody reads), so
  // that no register the transform reuses waits on the late loads
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
  if (early) {
#pragma unroll
    for (int i = 0; i < PF; ++i) {
      const int idx = tid + i * nthr;
      if (idx < n_late) {
        if constexpr (LATE_Y) pf[i] = load_y(idx);
        else pf[i] = load_z(idx);
      }
    }
  }
  __syncthreads();
  if ((MODE == LAT_FWD_MEAS || MODE == LAT_NORMAL || MODE == LAT_RESID) && pair && !half) {
    pack_real_pairs(lds, H, rs, L, tid, nthr);
    __syncthreads();
  }

  if (a.inverse) fft_rows_sized<ONE, true, OCT_CT_LAT_SIZES>(lds, nrow_t, rs, a.fd, twl, tid, nthr);
  else fft_rows_sized<ONE, false, OCT_CT_LAT_SIZES>(lds, nrow_t, rs, a.fd, twl, tid, nthr);

  if (MODE == LAT_FFT || MODE == LAT_ADJ_MEAS) {
    const int nout = (MODE == LAT_ADJ_MEAS && half) ? Lh * T : n;   // spectra of real rows: l <= L/2 suffices
    for (int idx = tid; idx < nout; idx += nthr) {
      const int l = idx >> lt, t = idx & (T - 1);
      if (t < nr) {
        const float2 v = (MODE == LAT_ADJ_MEAS && pair) ? unpack_real_pair(lds, rs, L, H, t, l) : lds[t * rs + l];
        a.dst[hbase + (int64_t)l * lg.es + t] = cscale(v, a.scale);
      }
    }
    return;
  }
  if (MODE == LAT_FWD_MEAS) {
    batched_for(n, tid, nthr,
      [&](int idx) { const int l = idx >> lt, t = min(idx & (T - 1), nr - 1); return mword(l, r0 + t); },
      [&](int idx, uint32_t m) {
        const int l = idx >> lt, t = idx & (T - 1);
        if (t < nr) {
          const float re = !pair ? lds[t * rs + l].x : (t < H ? lds[t * rs + l].x : lds[(t - H) * rs + l].y);
          const float yv = ((m >> ((r0 + t) & 31)) & 1u) ? re * a.scale : 0.f;
          a.dstf[base + (int64_t)l * lg.es + t] = yv;
        }
      });
    return;
  }
  if constexpr (MODE == LAT_UPDATE) {
    late_for(load_z,
      [&](int idx, Z2 v) {
        const int l = idx >> lt, t = idx & (T - 1);
        if (t < nr) {
          const float2 g = cscale(lds[t * rs + l], a.scale);
          const float xr = v.a.x + a.mu * (v.a.x - v.b.x), xi = v.a.y + a.mu * (v.a.y - v.b.y);
          a.dst[base + (int64_t)l * lg.es + t] = make_float2(xr - a.delta * g.x, xi - a.delta * g.y);
        }
      });
    return;
  }
  if (MODE == LAT_RESID) {
    // residual rows only (pairs: rows p and p + H from the real and imaginary parts of row p)
    double acc = 0.0;
    batched_for(n, tid, nthr,
      [&](int idx) { const int l = idx >> lt, t = min(idx & (T - 1), nr - 1);
                     return FM{a.y ? a.y[goff(idx)] : 0.f, mword(l, r0 + t)}; },
      [&](int idx, FM v) {
        const int l = idx >> lt, t = idx & (T - 1);
        if (t < nr) {
          const float re = !pair ? lds[t * rs + l].x : (t < H ? lds[t * rs + l].x : lds[(t - H) * rs + l].y);
          float r = 0.f;
          if ((v.m >> ((r0 + t) & 31)) & 1u) r = re * a.scale - v.f;
          acc += (double)r * (double)r;
          a.dstf[base + (int64_t)l * lg.es + t] = r;
        }
      });
    if (a.partial) {
      const double s = block_sum_d(acc, red);
      if (tid == 0) a.partial[bid] = s;
    }
    return;
  }
  if constexpr (MODE == LAT_NORMAL) if (pair) {
    // residual of rows p and p + H from the real and imaginary parts of row p
    double acc = 0.0;
    late_for(load_y,
      [&](int idx, YM v) {
        const int l = idx >> log2H, p = idx & (H - 1);
        const float2 vv = lds[p * rs + l];
        float ra = 0.f, rb = 0.f;
        if (p < nr && ((v.ma >> ((r0 + p) & 31)) & 1u)) ra = vv.x * a.scale - v.ya;
        if (p + H < nr && ((v.mb >> ((r0 + p + H) & 31)) & 1u)) rb = vv.y * a.scale - v.yb;
        if (a.partial) {
          acc += (double)ra * (double)ra;
          acc += (double)rb * (double)rb;
        }
        lds[p * rs + l] = make_float2(ra, rb);
      });
    __syncthreads();
    fft_rows_sized<ONE, false, OCT_CT_LAT_SIZES>(lds, H, rs, a.fd, twl, tid, nthr);
    for (int idx = tid; idx < (half ? Lh * T : n); idx += nthr) {
      const int l = idx >> lt, t = idx & (T - 1);
      if (t < nr) a.dst[hbase + (int64_t)l * lg.es + t] = cscale(unpack_real_pair(lds, rs, L, H, t, l), a.scale2);
    }
    if (a.partial) {   // the residual norm only when the caller asks for it
      const double s = block_sum_d(acc, red);
      if (tid == 0) a.partial[bid] = s;
    }
    return;
  }
  if (MODE == LAT_NORMAL) {
    double acc = 0.0;
    batched_for(n, tid, nthr,
      [&](int idx) { const int l = idx >> lt, t = min(idx & (T - 1), nr - 1);
                     return FM{a.y ? a.y[goff(idx)] : 0.f, mword(l, r0 + t)}; },
      [&](int idx, FM v) {
        const int l = idx >> lt, t = idx & (T - 1);
        float r = 0.f;
        if (t < nr && ((v.m >> ((r0 + t) & 31)) & 1u)) r = lds[t * rs + l].x * a.scale - v.f;
        acc += (double)r * (double)r;
        lds[t * rs + l] = make_float2(r, 0.f);
      });
    __syncthreads();
    fft_rows_sized<ONE, false, OCT_CT_LAT_SIZES>(lds, T, rs, a.fd, twl, tid, nthr);
    for (int idx = tid; idx < (half ? Lh * T : n); idx += nthr) {
      const int l = idx >> lt, t = idx & (T - 1);
      if (t < nr) a.dst[hbase + (int64_t)l * lg.es + t] = cscale(lds[t * rs + l], a.scale2);
    }
    if (a.partial) {
      const double s = block_sum_d(acc, red);
      if (tid == 0) a.partial[bid] = s;
    }
    return;
  }
  if constexpr (MODE == LAT_UPDATE_L1) {
    double acc = 0.0;
    late_for(load_z,
      [&](int idx, Z2 v) {
        const int l = idx >> lt, t = idx & (T - 1);
        float2 xn = make_float2(0.f, 0.f);
        if (t < nr) {
          const int64_t off = base + (int64_t)l * lg.es + t;
          const float2 g = cscale(lds[t * rs + l], a.scale);
          const float2 z = v.a, zo = v.b;
          const float vr = z.x + a.mu * (z.x - zo.x) - a.delta * g.x;
          const float vi = z.y + a.mu * (z.y - zo.y) - a.delta * g.y;
          const float mag = sqrtf(vr * vr + vi * vi);
          const float sc = mag > a.tau ? fminf(1.f - a.tau / mag, a.bound / mag) : 0.f;
          float2 zn;
          {
            // z^k and the next x from the rounded z^k (no fused multiply-adds across
            // the rounding): the same bits a resumed solve forms from stored z^k
#pragma clang fp contract(off)
            zn = make_float2(vr * sc, vi * sc);
            xn = make_float2(zn.x + a.mu_next * (zn.x - z.x), zn.y + a.mu_next * (zn.y - z.y));
          }
          acc += (double)sqrtf(zn.x * zn.x + zn.y * zn.y);
          a.zo[off] = zn;
        }
        lds[t * rs + l] = xn;
      });
    __syncthreads();
    fft_rows_sized<ONE, false, OCT_CT_LAT_SIZES>(lds, T, rs, a.fd, twl, tid, nthr);
    for (int idx = tid; idx < n; idx += nthr) {
      const int l = idx >> lt, t = idx & (T - 1);
      if (t < nr) a.dst[base + (int64_t)l * lg.es + t] = lds[t * rs + l];
    }
    if (a.partial) {
      const double s = block_sum_d(acc, red);
      if (tid == 0) a.partial[bid] = s;
    }
    return;
  }
}

}  // namespace

// Rows per tile and threads per block: the tile (T rows of L complex) stays
// within 64 KB of LDS and every FFT stage fits 2 butterflies per thread.
int lateral_pick_tile(const LineGeom& lg, const FftDesc& fd, int* nthr, int* rowstride) {
  const int rs = (lg.L % 2 == 0) ? lg.L + 1 : lg.L;  // odd stride spreads LDS banks
  const int mb = fft_maxb(fd);
  const int64_t budget = 65280;   // tile within 64 KB
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

template <int MODE, bool ONE>
hipError_t launch_lateral_m(const LatArgs& a, int nthr, hipStream_t s) {
  const size_t lds = ((size_t)lat_tile_f2(a.T, a.rowstride) + (size_t)a.fd.tw_total) * sizeof(float2);
  if (lds > 64 * 1024) {
    // once per instantiation (thread-safe initialisation of a local static)
    static const hipError_t set = hipFuncSetAttribute(reinterpret_cast<const void*>(&lat_kernel<MODE, ONE>),
                                                      hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 2048);
    if (set != hipSuccess) return set;
  }
  hipLaunchKernelGGL((lat_kernel<MODE, ONE>), dim3((a.lg.n_lines * a.n_tiles + 7) & ~7), dim3(nthr), lds, s, a);
  return hipGetLastError();
}

template <bool ONE>
hipError_t launch_lateral_t(LatMode mode, const LatArgs& a, int nthr, hipStream_t s) {
  switch (mode) {
    case LAT_FFT: return launch_lateral_m<LAT_FFT, ONE>(a, nthr, s);
    case LAT_FWD_MEAS: return launch_lateral_m<LAT_FWD_MEAS, ONE>(a, nthr, s);
    case LAT_ADJ_MEAS: return launch_lateral_m<LAT_ADJ_MEAS, ONE>(a, nthr, s);
    case LAT_NORMAL: return launch_lateral_m<LAT_NORMAL, ONE>(a, nthr, s);
    case LAT_UPDATE: return launch_lateral_m<LAT_UPDATE, ONE>(a, nthr, s);
    case LAT_UPDATE_L1: return launch_lateral_m<LAT_UPDATE_L1, ONE>(a, nthr, s);
    case LAT_RESID: return launch_lateral_m<LAT_RESID, ONE>(a, nthr, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_lateral(LatMode mode, const LatArgs& a, hipStream_t s) {
  const int64_t bf = (int64_t)a.T * (a.fd.n / a.fd.min_radix);
  const int mb = fft_maxb(a.fd);
  int nthr = 256;
  while (nthr < 1024 && bf > (int64_t)mb * nthr) nthr <<= 1;
  if (bf > (int64_t)mb * nthr) return hipErrorInvalidConfiguration;
  return fft_one(a.fd, a.T, nthr) ? launch_lateral_t<true>(mode, a, nthr, s)
                                  : launch_lateral_t<false>(mode, a, nthr, s);
}
