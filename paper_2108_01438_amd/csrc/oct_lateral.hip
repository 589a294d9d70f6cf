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

#include <type_traits>

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
  uint32_t m;   // the mask word of both rows
};

// float2 slots of the tile in LDS, rounded up to keep the twiddle rows that
// follow it 16-byte aligned
__host__ __device__ inline int lat_tile_f2(int T, int rs) { return (T * rs + 1) & ~1; }

// Offset of a tile element from the tile's origin.  OFF32 (the tile spans
// less than 4 GiB): a 32-bit byte offset of the float2 element (a float
// array takes half of it), made opaque at each access so that the access
// takes the uniform origin from scalar registers plus this one 32-bit
// register; otherwise a 64-bit element offset.
template <bool OFF32> struct LatOff;
template <> struct LatOff<true> {
  using type = uint32_t;
  __device__ static type of(int64_t elems) { return (uint32_t)(elems * 8); }
  template <typename T> __device__ static T* at(T* origin, type o) {
    uint32_t b = sizeof(T) == sizeof(float2) ? o : (o >> 1);
    asm volatile("" : "+v"(b));
    using C = std::conditional_t<std::is_const<T>::value, const char, char>;
    return reinterpret_cast<T*>(reinterpret_cast<C*>(origin) + b);
  }
};
template <> struct LatOff<false> {
  using type = int64_t;
  __device__ static type of(int64_t elems) { return elems; }
  template <typename T> __device__ static T* at(T* origin, type o) { return origin + o; }
};

template <int MODE, bool ONE, bool OFF32>
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
  // x lines whose source or destination has its own line stride (a volume's
  // padded spectral buffer on one side, an image on the other)
  const int64_t base_in = (lg.ocnt == 1 && a.sa_in) ? (int64_t)line * a.sa_in + r0 : base;
  const int64_t base_out = (lg.ocnt == 1 && a.sa_out) ? (int64_t)line * a.sa_out + r0 : base;
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
  // Element mapping.  nthr is a multiple of T, so thread tid owns one tile
  // row, t_own = tid mod T, and the laterals l = l_own + u LS (u = 0, 1, ...):
  // its row, clamped row and LDS row are fixed, and the offset of its next
  // element is the last one plus a uniform step.  Rows past the image
  // (ragged last tile) load a clamped valid row and store nothing.  The
  // real-pair loops run over rows p < H the same way (p_own = tid mod H).
  const int t_own = tid & (T - 1);
  const int l_own = tid >> lt;
  const int LS = nthr >> lt;
  const int t_cl = min(t_own, nr - 1);
  const bool t_ok = t_own < nr;
  const int log2H = lt > 0 ? lt - 1 : 0;
  const int p_own = tid & (H > 0 ? H - 1 : 0);
  const int l_ownH = tid >> log2H;
  const int LSH = nthr >> log2H;
  // per-array tile origins (uniform: scalar registers)
  auto org = [](auto* p, int64_t b) { return p ? p + b : p; };
  const float2* __restrict__ src_o = org(a.src, base_in);
  const float2* __restrict__ srch_o = org(a.src, half ? hbase : base_in);
  const float* __restrict__ srcf_o = org(a.srcf, base);
  const float2* __restrict__ z_o = org(a.z, base);
  const float2* __restrict__ zo_o = org(a.zo, base);
  float2* __restrict__ zow_o = org(a.zo, base);
  float2* __restrict__ xout_o = org(a.xout, base);
  float2* __restrict__ dst_o = org(a.dst, base_out);
  float2* __restrict__ dsth_o = org(a.dst, half ? hbase : base_out);
  float* __restrict__ dstf_o = org(a.dstf, base);
  const float* __restrict__ y_o = org(a.y, base);
  // mask words of this tile's rows (T <= 32 rows from a multiple of T: one word)
  const uint32_t* __restrict__ mrow = a.mask ? a.mask + (int64_t)latb * a.mask_words + (r0 >> 5) : nullptr;
  auto mword = [&](int mo) -> uint32_t { return mrow ? mrow[mo] : ~0u; };
  auto mbit = [&](uint32_t m, int t) -> bool { return (m >> ((r0 + t) & 31)) & 1u; };
  using Off = typename LatOff<OFF32>::type;

  // use(l, o, v) for the thread's laterals l = l_start + u lstep < Lend, with
  // o the offset of element (l, row) from the tile origin and
  // v = load(l, o, mo), mo = l mask_words; U loads in flight before the first use
  auto row_for = [&](int l_start, int lstep, int Lend, int row, auto load, auto use) __attribute__((always_inline)) {
    constexpr int U = 8;
    const Off os = LatOff<OFF32>::of((int64_t)lstep * lg.es);
    const int ms = lstep * a.mask_words;
    Off o = LatOff<OFF32>::of((int64_t)l_start * lg.es + row);
    int mo = l_start * a.mask_words;
    for (int lb = l_start; lb < Lend; lb += U * lstep, o += U * os, mo += U * ms) {
      using R = decltype(load(0, o, 0));
      R r[U];
      if (lb + (U - 1) * lstep < Lend) {   // the whole chunk (the usual case: no per-element branches)
#pragma unroll
        for (int u = 0; u < U; ++u) r[u] = load(lb + u * lstep, o + u * os, mo + u * ms);
#pragma unroll
        for (int u = 0; u < U; ++u) use(lb + u * lstep, o + u * os, r[u]);
      } else {
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (lb + u * lstep < Lend) r[u] = load(lb + u * lstep, o + u * os, mo + u * ms);
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (lb + u * lstep < Lend) use(lb + u * lstep, o + u * os, r[u]);
      }
    }
  };
  // the thread's laterals without loads: f(l, o)
  auto lat_each = [&](int l_start, int lstep, int Lend, int row, auto f) __attribute__((always_inline)) {
    const Off os = LatOff<OFF32>::of((int64_t)lstep * lg.es);
    Off o = LatOff<OFF32>::of((int64_t)l_start * lg.es + row);
    for (int l = l_start; l < Lend; l += lstep, o += os) f(l, o);
  };
  auto at = [&](auto* origin, Off o) __attribute__((always_inline)) { return LatOff<OFF32>::at(origin, o); };

  // Loads consumed after the transform (the extrapolated point, or the
  // iterate pair z, z_prev it comes from, of the gradient step; the data and
  // mask of the normal seam).  When they fit
  // PF per thread they are issued right after the tile's own loads and stream
  // in while the tile is transformed (load counters retire in order, so they
  // must come after every load the transform waits for).
  constexpr bool LATE_Z = MODE == LAT_UPDATE || MODE == LAT_UPDATE_L1;
  constexpr bool LATE_Y = MODE == LAT_NORMAL;
  constexpr int PF = 8;
  auto load_z = [&](int, Off o, int) { return Z2{*at(z_o, o), a.zo ? *at(zo_o, o) : make_float2(0.f, 0.f)}; };
  // rows p and p + H share their mask word; o is the offset of (l, row pa)
  const int pa = min(p_own, nr - 1), pb = min(p_own + H, nr - 1);
  const Off pbo = LatOff<OFF32>::of(pb - pa);
  auto load_y = [&](int, Off o, int mo) {
    return YM{a.y ? *at(y_o, o) : 0.f, a.y ? *at(y_o, o + pbo) : 0.f, mword(mo)};
  };
  using Late = std::conditional_t<LATE_Y, YM, Z2>;
  const int n_late = LATE_Y ? (n >> 1) : n;
  const bool early = (LATE_Z || (LATE_Y && pair)) && n_late <= PF * nthr;
  const int late_l0 = LATE_Y ? l_ownH : l_own, late_ls = LATE_Y ? LSH : LS, late_row = LATE_Y ? pa : t_cl;
  Late pf[PF];
  // run use(l, o, value) over the late elements, prefetched or loaded now
  auto late_for = [&](auto load, auto use) __attribute__((always_inline)) {
    if (early) {
      const Off os = LatOff<OFF32>::of((int64_t)late_ls * lg.es);
      const Off o0 = LatOff<OFF32>::of((int64_t)late_l0 * lg.es + late_row);
#pragma unroll
      for (int u = 0; u < PF; ++u) {
        const int l = late_l0 + u * late_ls;
        if (l < L) use(l, o0 + u * os, pf[u]);
      }
    } else {
      row_for(late_l0, late_ls, L, late_row, load, use);
    }
  };

  // ---- load the tile: element (row t, lateral l) -> lds[t * rs + l]
  if (MODE == LAT_ADJ_MEAS) {
    // real rows; paired: row t -> component t >= H of row t mod H
    float* ldsf = reinterpret_cast<float*>(lds);
    row_for(l_own, LS, L, t_cl,
      [&](int, Off o, int mo) { return FM{*at(srcf_o, o), mword(mo)}; },
      [&](int l, Off, FM v) {
        const float r = (t_ok && mbit(v.m, t_own)) ? v.f : 0.f;
        if (pair) ldsf[2 * ((t_own < H ? t_own : t_own - H) * rs + l) + (t_own < H ? 0 : 1)] = r;
        else lds[t_own * rs + l] = make_float2(r, 0.f);
      });
  } else if (MODE == LAT_FFT && a.z != nullptr) {
    row_for(l_own, LS, L, t_cl,
      [&](int, Off o, int) { return Z2{*at(z_o, o), *at(zo_o, o)}; },
      [&](int l, Off o, Z2 v) {
        float2 x;
        {
          // x = z + mu (z - z_prev) rounded step by step, as the fused l1 update
          // forms it: a resumed solve then matches an uninterrupted one bitwise
#pragma clang fp contract(off)
          x = make_float2(v.a.x + a.mu * (v.a.x - v.b.x), v.a.y + a.mu * (v.a.y - v.b.y));
        }
        lds[t_own * rs + l] = t_ok ? x : make_float2(0.f, 0.f);
        if (a.xout && t_ok) *at(xout_o, o) = x;
      });
  } else if ((MODE == LAT_FWD_MEAS || MODE == LAT_NORMAL) && half) {
    // half rows of Hermitian spectra, extended: row[L - l] = conj(row[l]); at
    // l = 0 (and L/2) only the real part belongs to the Hermitian row.
    // Paired: row p <- row_p + j row_{p+H}, so that one inverse transform
    // gives the real rows p and p + H (in .x and .y).
    if (pair) {
      row_for(l_ownH, LSH, Lh, pa,
        [&](int, Off o, int) { return Z2{*at(srch_o, o), *at(srch_o, o + pbo)}; },
        [&](int l, Off, Z2 v) {
          float2 va = p_own < nr ? v.a : make_float2(0.f, 0.f), vb = p_own + H < nr ? v.b : make_float2(0.f, 0.f);
          const bool self = l == 0 || 2 * l == L;
          if (self) { va.y = 0.f; vb.y = 0.f; }
          float2* ra = lds + p_own * rs;
          ra[l] = make_float2(va.x - vb.y, va.y + vb.x);
          if (!self) ra[L - l] = make_float2(va.x + vb.y, vb.x - va.y);
        });
    } else {
      row_for(l_own, LS, Lh, t_cl,
        [&](int, Off o, int) { return *at(srch_o, o); },
        [&](int l, Off, float2 v) {
          if (!t_ok) v = make_float2(0.f, 0.f);
          const bool self = l == 0 || 2 * l == L;
          if (self) v.y = 0.f;
          lds[t_own * rs + l] = v;
          if (!self) lds[t_own * rs + L - l] = cconj(v);
        });
    }
  } else {
    row_for(l_own, LS, L, t_cl,
      [&](int, Off o, int) { return *at(src_o, o); },
      [&](int l, Off, float2 v) { lds[t_own * rs + l] = t_ok ? v : make_float2(0.f, 0.f); });
  }
  // retire the tile's loads (including the clamped ones nobody reads), so
  // that no register the transform reuses waits on the late loads
  __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
  if (early) {
    const Off os = LatOff<OFF32>::of((int64_t)late_ls * lg.es);
    const Off o0 = LatOff<OFF32>::of((int64_t)late_l0 * lg.es + late_row);
    const int ms = late_ls * a.mask_words;
#pragma unroll
    for (int u = 0; u < PF; ++u) {
      const int l = late_l0 + u * late_ls;
      if (l < L) {
        const int mo = late_l0 * a.mask_words + u * ms;
        if constexpr (LATE_Y) pf[u] = load_y(l, o0 + u * os, mo);
        else pf[u] = load_z(l, o0 + u * os, mo);
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
    const int Lout = (MODE == LAT_ADJ_MEAS && half) ? Lh : L;   // spectra of real rows: l <= L/2 suffices
    if (t_ok)
      lat_each(l_own, LS, Lout, t_own, [&](int l, Off o) {
        const float2 v = (MODE == LAT_ADJ_MEAS && pair) ? unpack_real_pair(lds, rs, L, H, t_own, l)
                                                         : lds[t_own * rs + l];
        *at(dsth_o, o) = cscale(v, a.scale);
      });
    return;
  }
  if (MODE == LAT_FWD_MEAS) {
    row_for(l_own, LS, L, t_cl,
      [&](int, Off, int mo) { return mword(mo); },
      [&](int l, Off o, uint32_t m) {
        if (t_ok) {
          const float re = !pair ? lds[t_own * rs + l].x
                                 : (t_own < H ? lds[t_own * rs + l].x : lds[(t_own - H) * rs + l].y);
          *at(dstf_o, o) = mbit(m, t_own) ? re * a.scale : 0.f;
        }
      });
    return;
  }
  if constexpr (MODE == LAT_UPDATE) {
    late_for(load_z,
      [&](int l, Off o, Z2 v) {
        if (t_ok) {
          const float2 gr = cscale(lds[t_own * rs + l], a.scale);
          const float xr = v.a.x + a.mu * (v.a.x - v.b.x), xi = v.a.y + a.mu * (v.a.y - v.b.y);
          *at(dst_o, o) = make_float2(xr - a.delta * gr.x, xi - a.delta * gr.y);
        }
      });
    return;
  }
  if (MODE == LAT_RESID) {
    // residual rows only (pairs: rows p and p + H from the real and imaginary parts of row p)
    double acc = 0.0;
    row_for(l_own, LS, L, t_cl,
      [&](int, Off o, int mo) { return FM{a.y ? *at(y_o, o) : 0.f, mword(mo)}; },
      [&](int l, Off o, FM v) {
        if (t_ok) {
          const float re = !pair ? lds[t_own * rs + l].x
                                 : (t_own < H ? lds[t_own * rs + l].x : lds[(t_own - H) * rs + l].y);
          float r = 0.f;
          if (mbit(v.m, t_own)) r = re * a.scale - v.f;
          acc += (double)r * (double)r;
          *at(dstf_o, o) = r;
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
    const bool pa_ok = p_own < nr, pb_ok = p_own + H < nr;
    late_for(load_y,
      [&](int l, Off, YM v) {
        const float2 vv = lds[p_own * rs + l];
        float ra = 0.f, rb = 0.f;
        if (pa_ok && mbit(v.m, p_own)) ra = vv.x * a.scale - v.ya;
        if (pb_ok && mbit(v.m, p_own + H)) rb = vv.y * a.scale - v.yb;
        if (a.partial) {
          acc += (double)ra * (double)ra;
          acc += (double)rb * (double)rb;
        }
        lds[p_own * rs + l] = make_float2(ra, rb);
      });
    __syncthreads();
    fft_rows_sized<ONE, false, OCT_CT_LAT_SIZES>(lds, H, rs, a.fd, twl, tid, nthr);
    if (t_ok)
      lat_each(l_own, LS, half ? Lh : L, t_own, [&](int l, Off o) {
        *at(dsth_o, o) = cscale(unpack_real_pair(lds, rs, L, H, t_own, l), a.scale2);
      });
    if (a.partial) {   // the residual norm only when the caller asks for it
      const double s = block_sum_d(acc, red);
      if (tid == 0) a.partial[bid] = s;
    }
    return;
  }
  if (MODE == LAT_NORMAL) {
    double acc = 0.0;
    row_for(l_own, LS, L, t_cl,
      [&](int, Off o, int mo) { return FM{a.y ? *at(y_o, o) : 0.f, mword(mo)}; },
      [&](int l, Off, FM v) {
        float r = 0.f;
        if (t_ok && mbit(v.m, t_own)) r = lds[t_own * rs + l].x * a.scale - v.f;
        acc += (double)r * (double)r;
        lds[t_own * rs + l] = make_float2(r, 0.f);
      });
    __syncthreads();
    fft_rows_sized<ONE, false, OCT_CT_LAT_SIZES>(lds, T, rs, a.fd, twl, tid, nthr);
    if (t_ok)
      lat_each(l_own, LS, half ? Lh : L, t_own, [&](int l, Off o) {
        *at(dsth_o, o) = cscale(lds[t_own * rs + l], a.scale2);
      });
    if (a.partial) {
      const double s = block_sum_d(acc, red);
      if (tid == 0) a.partial[bid] = s;
    }
    return;
  }
  if constexpr (MODE == LAT_UPDATE_L1) {
    double acc = 0.0;
    late_for(load_z,
      [&](int l, Off o, Z2 v) {
        float2 xn = make_float2(0.f, 0.f);
        if (t_ok) {
          const float2 gr = cscale(lds[t_own * rs + l], a.scale);
          const float2 z = v.a, zo = v.b;
          const float vr = z.x + a.mu * (z.x - zo.x) - a.delta * gr.x;
          const float vi = z.y + a.mu * (z.y - zo.y) - a.delta * gr.y;
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
          *at(zow_o, o) = zn;
        }
        lds[t_own * rs + l] = xn;
      });
    __syncthreads();
    fft_rows_sized<ONE, false, OCT_CT_LAT_SIZES>(lds, T, rs, a.fd, twl, tid, nthr);
    if (t_ok)
      lat_each(l_own, LS, L, t_own, [&](int l, Off o) { *at(dst_o, o) = lds[t_own * rs + l]; });
    if (a.partial) {
      const double s = block_sum_d(acc, red);
      if (tid == 0) a.partial[bid] = s;
    }
    return;
  }
}

}  // namespace

// Rows per tile and threads per block: the tile (T rows of L complex) stays
// within 64 KB of LDS and every FFT stage fits 2 butterflies per thread; on
// images too small to give every CU a tile, the tiles narrow (to two rows at
// least) until they do.
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
        // small images: narrower tiles while the largest would leave CUs
        // without a tile (the pass is then one tile's chain long, and a
        // narrower tile's chain is shorter); down to row pairs
        while (T > 2 && (int64_t)lg.n_lines * ((lg.rows + T - 1) / T) < 256) T >>= 1;
        *nthr = nt;
        *rowstride = rs;
        return T;
      }
    }
  }
  return 0;
}

template <int MODE, bool ONE, bool OFF32>
hipError_t launch_lateral_m(const LatArgs& a, int nthr, hipStream_t s) {
  const size_t lds = ((size_t)lat_tile_f2(a.T, a.rowstride) + (size_t)a.fd.tw_total) * sizeof(float2);
  if (lds > 64 * 1024) {
    // once per instantiation (thread-safe initialisation of a local static)
    static const hipError_t set = hipFuncSetAttribute(reinterpret_cast<const void*>(&lat_kernel<MODE, ONE, OFF32>),
                                                      hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024 - 2048);
    if (set != hipSuccess) return set;
  }
  hipLaunchKernelGGL((lat_kernel<MODE, ONE, OFF32>), dim3((a.lg.n_lines * a.n_tiles + 7) & ~7), dim3(nthr), lds, s,
                     a);
  return hipGetLastError();
}

template <bool ONE, bool OFF32>
hipError_t launch_lateral_t(LatMode mode, const LatArgs& a, int nthr, hipStream_t s) {
  switch (mode) {
    case LAT_FFT: return launch_lateral_m<LAT_FFT, ONE, OFF32>(a, nthr, s);
    case LAT_FWD_MEAS: return launch_lateral_m<LAT_FWD_MEAS, ONE, OFF32>(a, nthr, s);
    case LAT_ADJ_MEAS: return launch_lateral_m<LAT_ADJ_MEAS, ONE, OFF32>(a, nthr, s);
    case LAT_NORMAL: return launch_lateral_m<LAT_NORMAL, ONE, OFF32>(a, nthr, s);
    case LAT_UPDATE: return launch_lateral_m<LAT_UPDATE, ONE, OFF32>(a, nthr, s);
    case LAT_UPDATE_L1: return launch_lateral_m<LAT_UPDATE_L1, ONE, OFF32>(a, nthr, s);
    case LAT_RESID: return launch_lateral_m<LAT_RESID, ONE, OFF32>(a, nthr, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_lateral(LatMode mode, const LatArgs& a, hipStream_t s) {
  const int64_t bf = (int64_t)a.T * (a.fd.n / a.fd.min_radix);
  const int mb = fft_maxb(a.fd);
  int nthr = 256;
  while (nthr < 1024 && bf > (int64_t)mb * nthr) nthr <<= 1;
  if (bf > (int64_t)mb * nthr) return hipErrorInvalidConfiguration;
  // a thread owns one tile row: the threads must be a multiple of the rows
  if (nthr % a.T != 0) return hipErrorInvalidConfiguration;
  // 32-bit byte offsets inside a tile when its span (lateral stride times the
  // laterals, plus the rows) stays below 4 GiB
  const bool off32 = ((int64_t)(a.lg.L - 1) * a.lg.es + a.T) * (int64_t)sizeof(float2) < ((int64_t)1 << 32);
  if (fft_one(a.fd, a.T, nthr))
    return off32 ? launch_lateral_t<true, true>(mode, a, nthr, s) : launch_lateral_t<true, false>(mode, a, nthr, s);
  return off32 ? launch_lateral_t<false, true>(mode, a, nthr, s) : launch_lateral_t<false, false>(mode, a, nthr, s);
}
