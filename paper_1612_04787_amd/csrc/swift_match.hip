// Whitened FFT window matching: the batched forward path.
//
// Method (Wetzel et al., arXiv 1612.04787, Section III): each window pair is
// apodized with a cosine taper, correlated in the frequency domain with the
// Fourier amplitudes scaled by a power p in [0, 1] (0 = plain correlation,
// 1 = phase-only), transformed back, and scored by the Z-score of its peak.
//
// Per pair the two real windows a, b travel together as one complex field
// z = a'T + i b'T (a' = a - offset, T the separable taper), so the forward 2-D
// transform is a single complex FFT.  Five kernels per window size N:
//   k_row_fwd   gather (bilinear affine, uint8/fp32 -> fp32), taper, row FFTs,
//               per-slice sums; writes the row spectra in tiles of 8 rows
//               ([y/8][kx][y%8], see ztile), one contiguous region per block.
//   k_pair_stats  reduces the sums to the weighted means and eps^2.
//   k_col_pair  column FFTs of kx and N-kx, split into F_A and F_B, removes the
//               weighted mean in the spectrum (F -= m * tau(ky) tau(kx)),
//               whitens the cross power, inverse column FFT; writes in place
//               (one FFT group per column pair).
//   k_row_inv   inverse row FFTs (two real rows per complex FFT), per-slice
//               top-2 / argmax and FP64 sum, sum of squares; optional surface.
//               With a search radius r (the pruned inverse) only the row
//               blocks near the origin run, the peak is searched within
//               |shift| <= r, and the column pass supplies sum |C|^2 instead.
//   k_finalize  reduces the slices, recomputes the three rows around the peak
//               for the 3x3 centroid and writes the match record.
// Pearson mode runs the same kernels at p = 0 with window A cut to its
// central template (a box taper for the mean, unit taper for the gather),
// plus k_ncc_energy for the per-placement patch energies, and searches the
// Pearson coefficients c / sqrt(template energy x patch energy).
#include <float.h>
#include <limits.h>
#include <math.h>

#include "swift_dev.hpp"
#include "swift_tile.hpp"

namespace swift {

// ---------------------------------------------------------------- taper spectrum
// tau[k] = sum_i t(i) exp(-2 pi i k i / N) in FP64 from the same FP32 taper
// values the gather uses.  Since t = 1 outside the 2L edge samples,
// tau[k] = N [k == 0] - sum_{edge i} (1 - t(i)) exp(-2 pi i k i / N).
// Block 0 also writes sum t and sum t^2.  Each block first puts the n
// roots of unity and the 2L edge weights 1 - t(i) in LDS (the same values a
// per-term evaluation gives), so a bin costs 2L table reads.
__global__ void __launch_bounds__(256) k_taper(int n, int L, float2* __restrict__ tau, float* __restrict__ taper,
                                               TaperInfo* info) {
  __shared__ double red[2][4];
  __shared__ double wc[1024], ws[1024], om[1024];
  const int Le = min(L, n / 2);
  for (int m = threadIdx.x; m < n; m += blockDim.x) {
    double sn, cs;
    sincospi(2.0 * (double)m / (double)n, &sn, &cs);
    wc[m] = cs;
    ws[m] = sn;
  }
  for (int q = threadIdx.x; q < 2 * Le; q += blockDim.x) {
    const int i = q < Le ? q : n - 2 * Le + q;
    om[q] = 1.0 - (double)taper_at(i, n, L);
  }
  __syncthreads();
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) {
    taper[k] = taper_at(k, n, L);
    double re = (k == 0) ? (double)n : 0.0, im = 0.0;
    for (int q = 0; q < 2 * Le; ++q) {
      const int i = q < Le ? q : n - 2 * Le + q;
      const int m = (int)(((long long)k * i) % n);
      re -= om[q] * wc[m];
      im += om[q] * ws[m];
    }
    tau[k] = make_float2((float)re, (float)im);
  }
  if (blockIdx.x != 0) return;
  double s1 = 0.0, s2 = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double t = (double)taper_at(i, n, L);
    s1 += t;
    s2 += t * t;
  }
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
  if (ln == 0) {
    red[0][wv] = s1;
    red[1][wv] = s2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    TaperInfo ti;
    ti.sum_t = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    ti.sum_t2 = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    ti.L = L;
    ti.pad = 0;
    *info = ti;
  }
}

// Pearson tables: the gather runs with a unit taper, and the template of
// window A is the box [n/4, 3n/4) in both axes, so tau[k] = sum over the box
// of exp(-2 pi i k i / n) (FP64, the roots of unity tabled in LDS) and the
// taper sums are those of the box.
__global__ void __launch_bounds__(256) k_taper_box(int n, float2* __restrict__ tau, float* __restrict__ taper,
                                                   TaperInfo* info) {
  __shared__ double wc[1024], ws[1024];
  for (int j = threadIdx.x; j < n; j += blockDim.x) {
    double sn, cs;
    sincospi(2.0 * (double)j / (double)n, &sn, &cs);
    wc[j] = cs;
    ws[j] = sn;
  }
  __syncthreads();
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int m = n / 2, c0 = n / 4;
  if (k < n) {
    taper[k] = 1.0f;
    double re = 0.0, im = 0.0;
    for (int i = c0; i < c0 + m; ++i) {
      const int q = (int)(((long long)k * i) % n);
      re += wc[q];
      im -= ws[q];
    }
    tau[k] = make_float2((float)re, (float)im);
  }
  if (k == 0) {
    TaperInfo ti;
    ti.sum_t = (double)m;
    ti.sum_t2 = (double)m;
    ti.L = 0;
    ti.pad = 0;
    *info = ti;
  }
}

// ---------------------------------------------------------------- row pass (forward)
// Window samples of the forward row pass.  A thread covers ITER consecutive
// rows r0 + i of the slice (r0 = (tid / N) ITER) and XV columns: tid % N for
// N <= 256, the XV adjacent columns XV tid + c otherwise, so that one aligned
// tile read serves the bilinear pairs of several columns.
template <int N, int R>
struct FwdMap {
  static constexpr int XV = GatherCfg<N>::XV, RPI = GatherCfg<N>::RPI, ITER = R / RPI;
  __device__ static int col(int tid, int c) { return XV > 1 ? XV * tid + c : tid % N; }
  __device__ static int row0(int tid) { return RPI > 1 ? (tid / N) * ITER : 0; }
};

// LDS layout of the forward row pass.  When a thread's rows are the slice's
// rows (N >= 256) the source tile sits at the end of the stage instead of in
// an array of its own: stage rows [0, FL) lie below it and are written during
// the gather, rows [FL, R) overlap it and are held in registers until both
// images are gathered.  Less LDS per workgroup, more workgroups per CU.
template <int N, int R, int BUDGET>
struct FwdStage {
  static constexpr int RS = fwd_stride<N, R>();
  static constexpr int BYTES = R * RS * 8;
  static constexpr bool ALIAS = GatherCfg<N>::RPI == 1 && BUDGET > 0 && BUDGET + 4 + 16 <= BYTES;
  static constexpr int TOFF = ALIAS ? ((BYTES - BUDGET - 4) & ~15) : 0;  // tile offset, bytes (16-aligned)
  static constexpr int FL = ALIAS ? TOFF / (RS * 8) : R;                  // first row the tile overlaps
  static constexpr int NL = R - FL > 0 ? R - FL : 1;                      // late-row registers (at least 1)
};

// Gathers one image of the thread's samples into the stage (real parts for
// A, imaginary parts for B): a' T with a' = sample - o and T = t(x) t(y),
// formed as ((a - o) t(x)) t(y).  Adds the slice sum s2 = sum (a'T)^2 and,
// per column, s3c[c] = sum_r (a'T) t(y), so that sum (a'T) T =
// sum_c t(x_c) s3c[c].  (sum a'T is the DC bin of the row transforms.)
template <int N, int R, int FL, int NL, bool IM, bool TILE>
__device__ __forceinline__ void gather_rows(float2* __restrict__ stage, float (&late)[NL][GatherCfg<N>::XV],
                                            const uint32_t* __restrict__ tile, const TileGeom& g,
                                            const RowParam* __restrict__ rp, const float* __restrict__ trow,
                                            const float (&ku)[2][GatherCfg<N>::XV], const swift_image& im,
                                            bool border, const float (&tx)[GatherCfg<N>::XV], float o, int tid,
                                            float& s2, float (&s3c)[GatherCfg<N>::XV], bool& cl) {
  using M = FwdMap<N, R>;
  constexpr int XV = M::XV, ITER = M::ITER, RS = fwd_stride<N, R>();
  const int rowb = g.ts * 4;
  const gptr<unsigned char> base = to_global<unsigned char>(im.data);
  const int r0 = M::row0(tid);
  float* st = (float*)stage + (IM ? 1 : 0);
  // rows i < FL go to the stage, the others (only when rows are compile-time
  // indices, RPI == 1) to late[i - FL]
  constexpr int FLI = FL < ITER ? FL : ITER;
  auto row = [&](int i, auto sink) {
    const int r = r0 + i;
    const RowParam p = rp[r];
    const float ty = trow[r];
#pragma unroll
    for (int c = 0; c < XV; ++c) {
      const float xr = p.fx + ku[0][c], yr = p.fy + ku[1][c];
      const float xf = floorf(xr), yf = floorf(yr);
      const float fx = xr - xf, fy = yr - yf;
      const int x0 = p.bx + (int)xf, y0 = p.by + (int)yf;
      float i00, i10, i01, i11;
      if constexpr (TILE) {
        if (border) cl |= (x0 + g.xlo < 0) | (x0 + g.xlo > im.width - 2) | (y0 + g.ylo < 0) | (y0 + g.ylo > im.height - 2);
        const int ix = min(max(x0, 0), rowb - 2), iy = min(max(y0, 0), g.ht - 2);
        const int off = iy * rowb + ix;
        const uint32_t vt = tile_pair(tile, off), vb = tile_pair(tile, off + rowb);
        i00 = (float)(vt & 255u);
        i10 = (float)((vt >> 8) & 255u);
        i01 = (float)(vb & 255u);
        i11 = (float)((vb >> 8) & 255u);
      } else {
        cl |= (x0 < 0) | (x0 > im.width - 2) | (y0 < 0) | (y0 > im.height - 2);
        const int cx0 = min(max(x0, 0), im.width - 1), cx1 = min(max(x0 + 1, 0), im.width - 1);
        const int cy0 = min(max(y0, 0), im.height - 1), cy1 = min(max(y0 + 1, 0), im.height - 1);
        const gptr<unsigned char> r0p = base + (int64_t)cy0 * im.pitch;
        const gptr<unsigned char> r1p = base + (int64_t)cy1 * im.pitch;
        if (im.dtype == SWIFT_U8) {
          i00 = (float)r0p[cx0];
          i10 = (float)r0p[cx1];
          i01 = (float)r1p[cx0];
          i11 = (float)r1p[cx1];
        } else {
          i00 = ((gptr<float>)r0p)[cx0];
          i10 = ((gptr<float>)r0p)[cx1];
          i01 = ((gptr<float>)r1p)[cx0];
          i11 = ((gptr<float>)r1p)[cx1];
        }
      }
      // (1-fy)((1-fx) i00 + fx i10) + fy((1-fx) i01 + fx i11), in lerp form
      const float top = fmaf(fx, i10 - i00, i00), bot = fmaf(fx, i11 - i01, i01);
      const float val = fmaf(fy, bot - top, top);
      const float at = ((val - o) * tx[c]) * ty;
      s2 = fmaf(at, at, s2);
      s3c[c] = fmaf(at, ty, s3c[c]);
      sink(r, c, at);
    }
  };
#pragma unroll 2
  for (int i = 0; i < FLI; ++i) row(i, [&](int r, int c, float at) { st[2 * (r * RS + lidx(M::col(tid, c)))] = at; });
#pragma unroll
  for (int i = FLI; i < ITER; ++i) row(i, [&](int r, int c, float at) { late[r - FL][c] = at; });
}

// Gather of a translation window (identity linear part): every sample of the
// window has the same bilinear weights (fx, fy), so a thread walks down its
// columns and reuses the horizontal interpolation of each tile row for the
// next output row.  One aligned read of a tile row gives the bytes of two
// adjacent columns.  The offset enters the horizontal interpolation, h - o =
// fx (b1 - b0) + (b0 - o), so the samples of a constant window are exactly 0.
// p0: the sampling parameters of the thread's first row r0 (bx, by in tile
// coordinates; fx, fy the same on every row).  Same outputs and sums as
// gather_rows.
template <int N, int R, int FL, int NL, bool IM>
__device__ __forceinline__ void gather_rows_trans(float2* __restrict__ stage, float (&late)[NL][GatherCfg<N>::XV],
                                                  const uint32_t* __restrict__ tile, const TileGeom& g,
                                                  const RowParam& p0, const float* __restrict__ taper, int y0,
                                                  const swift_image& im, bool border,
                                                  const float (&tx)[GatherCfg<N>::XV], float o, int tid,
                                                  float& s2, float (&s3c)[GatherCfg<N>::XV], bool& cl) {
  using M = FwdMap<N, R>;
  constexpr int XV = M::XV, ITER = M::ITER, RS = fwd_stride<N, R>();
  constexpr int TS = 4 * tile_cw<N>();  // dwords between tile rows (tile_geom_trans)
  const int r0 = M::row0(tid);
  float* st = (float*)stage + (IM ? 1 : 0);
  const float fx = p0.fx, fy = p0.fy;  // the same for every row of the window
  // first column's byte in the tile row; the thread reads bytes ix .. ix + XV.
  // tile_geom_trans leaves a pixel of margin on every side, so rows p0.by ..
  // p0.by + ITER and these bytes lie inside the tile: no clamping
  const int ix = p0.bx + (M::col(tid, 0) - N / 2);
  // samples span columns ix .. ix + XV and rows p0.by .. p0.by + ITER (tile
  // coordinates), so one range test gives the clamp flag of all of them
  if (border)
    cl |= (ix + g.xlo < 0) | (ix + XV - 1 + g.xlo > im.width - 2) | (p0.by + g.ylo < 0) |
          (p0.by + ITER - 1 + g.ylo > im.height - 2);
  const uint32_t sh = (uint32_t)(ix & 3);
  // the thread's bytes of every row sit a constant TS dwords apart
  const uint32_t* wb = tile + p0.by * TS + (ix >> 2);
  auto hrow = [&](int i, float (&h)[XV]) {
    const uint32_t* w = wb + i * TS;
#pragma unroll
    for (int c = 0; c < XV; c += 2) {
      // bytes ix + c .. ix + c + 3
      const int oc = (int)sh + c;
      const uint32_t v = __builtin_amdgcn_alignbyte(w[(oc >> 2) + 1], w[oc >> 2], (uint32_t)(oc & 3));
      // the converted bytes go through an empty asm so that b1 - b0 is one
      // FP32 subtraction of values converted anyway, not an integer
      // difference converted again
      float b0 = (float)(v & 255u), b1 = (float)((v >> 8) & 255u);
      asm("" : "+v"(b0), "+v"(b1));
      h[c] = fmaf(fx, b1 - b0, b0 - o);
      if (c + 1 < XV) {
        float b2 = (float)((v >> 16) & 255u);
        asm("" : "+v"(b2));
        h[c + 1] = fmaf(fx, b2 - b1, b1 - o);
      }
    }
  };
  float h0[XV];
  hrow(0, h0);
  constexpr int FLI = FL < ITER ? FL : ITER;
  auto row = [&](int i, auto sink) {
    const int r = r0 + i;
    float h1[XV];
    hrow(i + 1, h1);
    const float ty = taper[y0 + r];
#pragma unroll
    for (int c = 0; c < XV; ++c) {
      const float val = fmaf(fy, h1[c] - h0[c], h0[c]);  // sample - o
      h0[c] = h1[c];
      const float at = (val * tx[c]) * ty;
      s2 = fmaf(at, at, s2);
      s3c[c] = fmaf(at, ty, s3c[c]);
      sink(r, c, at);
    }
  };
#pragma unroll
  for (int i = 0; i < FLI; ++i) row(i, [&](int r, int c, float at) { st[2 * (r * RS + lidx(M::col(tid, c)))] = at; });
#pragma unroll
  for (int i = FLI; i < ITER; ++i) row(i, [&](int r, int c, float at) { late[r - FL][c] = at; });
}

// Pearson mode, between the gather (unit taper) and the row FFTs: window A
// keeps only its central m x m template (m = N/2 from c0 = N/4) and its sums
// are taken over the template alone; every row of window B gives its sums of
// f' and f'^2 over the m columns of every placement j = sx + N/4 in [0, N/2]
// (prefix sums along the row: the row half of the cumulative-area
// correction).  One wave per stage row; lane l holds x = l + 64 e, so each
// segment of 64 columns is one wave scan and a placement's sum P(j + m) -
// P(j) reads two entries of one lane (at N = 64 the upper one is a lane
// 32 away).
template <int N, int R, int RS>
__device__ void pearson_rows(float2* __restrict__ stage, const MatchArgs& a, int pair, int y0, int tid,
                             float (&s)[6]) {
  constexpr int M = N / 2, C0 = N / 4, NP = N / 2 + 1, EL = N / 64;
  const int wv = tid >> 6, ln = tid & 63;
  s[0] = s[1] = 0.0f;
  for (int r = wv; r < R; r += 4) {
    float2* row = stage + r * RS;
    const int y = y0 + r;
    const bool yin = y >= C0 && y < C0 + M;
    float q1[EL], q2[EL];  // exclusive prefix sums at x = ln + 64 e
    float c1 = 0.0f, c2 = 0.0f;  // totals of the earlier segments
#pragma unroll
    for (int e = 0; e < EL; ++e) {
      const int x = ln + 64 * e;
      const float2 z = row[lidx(x)];
      if (yin && x >= C0 && x < C0 + M) {
        s[0] += z.x;
        s[1] = fmaf(z.x, z.x, s[1]);
      } else {
        row[lidx(x)] = make_float2(0.0f, z.y);
      }
      const float f = z.y, f2 = z.y * z.y;
      const float i1 = wave_incl_scan_f32(f), i2 = wave_incl_scan_f32(f2);
      q1[e] = c1 + (i1 - f);
      q2[e] = c2 + (i2 - f2);
      c1 += __int_as_float(__builtin_amdgcn_readlane(__float_as_int(i1), 63));
      c2 += __int_as_float(__builtin_amdgcn_readlane(__float_as_int(i2), 63));
    }
    float2* dst = a.ncc_rows + ((size_t)pair * N + y) * NP;
    if constexpr (EL == 1) {
      const float u1 = __shfl_down(q1[0], 32, 64), u2 = __shfl_down(q2[0], 32, 64);
      if (ln < 32) dst[ln] = make_float2(u1 - q1[0], u2 - q2[0]);
      if (ln == 32) dst[32] = make_float2(c1 - q1[0], c2 - q2[0]);
    } else {
#pragma unroll
      for (int k = 0; k < EL / 2; ++k) dst[ln + 64 * k] = make_float2(q1[k + EL / 2] - q1[k], q2[k + EL / 2] - q2[k]);
      if (ln == 0) dst[M] = make_float2(c1 - q1[EL / 2], c2 - q2[EL / 2]);
    }
  }
  s[2] = s[0];  // sum a' T^2 with a 0/1 template mask
}

// ---------------------------------------------------------------- per-pair geometry
// One thread per pair: the FP64 part of the window set-up that every row
// block of the pair would otherwise repeat (origin split, translation test,
// centre pixel).
__global__ void __launch_bounds__(256) k_pair_geom(MatchArgs a) {
  const int pair = blockIdx.x * 256 + threadIdx.x;
  if (pair >= a.npairs) return;
  const int kk[2] = {min(max(a.img_a[pair], 0), a.n_imgs - 1), min(max(a.img_b[pair], 0), a.n_imgs - 1)};
  const float* th[2] = {a.th_a + 8 * (size_t)pair, a.th_b + 8 * (size_t)pair};
  PairGeom pg;
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    swift_image im = a.imgs[kk[m]];
    im.width = max(im.width, 2);
    im.height = max(im.height, 2);
    const RowAffine ra = row_affine(th[m]);
    const bool trans = ra.a11 == 1.0 && ra.a12 == 0.0 && ra.a21 == 0.0 && ra.a22 == 1.0;
    const double X = fmin(fmax(ra.xc, -1e9), 1e9), Y = fmin(fmax(ra.yc, -1e9), 1e9);
    const double fxd = floor(X), fyd = floor(Y);
    WinGeom w;
    w.bx0 = (int)fxd;
    w.by0 = (int)fyd;
    w.fx = (float)(X - fxd);
    w.fy = (float)(Y - fyd);
    w.off = centre_pixel(im, ra);
    w.flags = (trans ? 1 : 0) | ((fabs(X) < 1e8 && fabs(Y) < 1e8) ? 2 : 0);
    pg.w[m] = w;
  }
  a.geom[pair] = pg;
}

// LDS of the forward row pass (one object per workgroup, shared by both
// variants of the body).
template <int N, int R, int BUDGET>
struct FwdLds {
  using SL = FwdStage<N, R, BUDGET>;
  __align__(16) float2 stage[R * SL::RS];
  // + 1: tile_pair reads the dword after a pair
  __align__(16) uint32_t tile_own[(BUDGET > 0 && !SL::ALIAS) ? BUDGET / 4 + 1 : 1];
  RowParam rparam[2][R];
  float trow[R];
  double red[4][6];
  int redc[4];
};

// Per-workgroup set-up of the two windows (image, affine, tile geometry,
// border test, translation test, first-row parameters of a translation).
struct FwdWin {
  swift_image im[2];
  RowAffine ra[2];
  TileGeom tg[2];
  RowParam pt[2];
  bool border[2], trans[2];
};

// Body of the forward row pass.  FAST: both windows are translations whose
// tiles are in use and lie inside their images (the common case), so the
// gather takes the constant-weight path with no clamping and no per-row
// parameters; the body is compiled once with these facts as constants and
// once for the general case.
template <int N, int R, int BUDGET, int TRW, bool PEARSON, bool FAST>
__device__ __forceinline__ void row_fwd_body(const MatchArgs& a, FwdLds<N, R, BUDGET>& sh, const FwdWin& wn,
                                             const PairGeom& pg, int pair, int slice, int y0, int tid) {
  using C = FftCfg<N>;
  constexpr int T = C::T, E = C::E, G = 256 / T, NSLICE = N / R;
  using SL = FwdStage<N, R, BUDGET>;
  constexpr int RS = SL::RS, FL = SL::FL, NL = SL::NL;
  constexpr int XV = GatherCfg<N>::XV;
  using M = FwdMap<N, R>;
  float2* const stage = sh.stage;
  uint32_t* const tile =
      SL::ALIAS ? reinterpret_cast<uint32_t*>(reinterpret_cast<char*>(sh.stage) + SL::TOFF) : sh.tile_own;
  const int g = tid / T, t = tid % T;
  const bool use0 = FAST || wn.tg[0].use, use1 = FAST || wn.tg[1].use;
  const bool tr0 = FAST || wn.trans[0], tr1 = FAST || wn.trans[1];
  const bool bd0 = !FAST && wn.border[0], bd1 = !FAST && wn.border[1];

  // all tile loads of both images in flight before anything waits on them
  uint4 bufA[TRW], bufB[TRW];
  if (use0) tile_fetch<tile_cw<N>()>(bufA, wn.tg[0], wn.im[0], tid);
  if (use1) tile_fetch<tile_cw<N>()>(bufB, wn.tg[1], wn.im[1], tid);
  if constexpr (!FAST) {
    // per-row parameters of the windows not gathered by translation from a
    // tile (lanes 0..2R-1 of wave 0) and row tapers (wave 1)
    if (tid < 2 * R && !(tid >= R ? (tr1 && use1) : (tr0 && use0))) {
      // image chosen by value selects (an index into the per-image arrays would
      // send them to per-lane scratch memory)
      const bool mb = tid >= R;
      const int r = tid % R;
      const int xo = mb ? (use1 ? wn.tg[1].xlo : 0) : (use0 ? wn.tg[0].xlo : 0);
      const int yo = mb ? (use1 ? wn.tg[1].ylo : 0) : (use0 ? wn.tg[0].ylo : 0);
      RowParam p;
      if (mb ? tr1 : tr0) {
        // a translation window's row r is its origin moved down by v rows
        const WinGeom& w = mb ? pg.w[1] : pg.w[0];
        p.bx = w.bx0 - xo;
        p.by = w.by0 + (y0 + r - N / 2) - yo;
        p.fx = w.fx;
        p.fy = w.fy;
      } else {
        const double xc = mb ? wn.ra[1].xc : wn.ra[0].xc, yc = mb ? wn.ra[1].yc : wn.ra[0].yc;
        const double a12 = mb ? wn.ra[1].a12 : wn.ra[0].a12, a22 = mb ? wn.ra[1].a22 : wn.ra[0].a22;
        const double v = (double)(y0 + r - N / 2);
        const double X = fmin(fmax(xc + a12 * v, -1e9), 1e9);
        const double Y = fmin(fmax(yc + a22 * v, -1e9), 1e9);
        const double bxd = floor(X), byd = floor(Y);
        p.bx = (int)bxd - xo;
        p.by = (int)byd - yo;
        p.fx = (float)(X - bxd);
        p.fy = (float)(Y - byd);
      }
      sh.rparam[mb ? 1 : 0][r] = p;
    }
    if (tid >= 64 && tid < 64 + R) sh.trow[tid - 64] = a.taper[y0 + tid - 64];
  }
  // the offsets: the centre pixels, the same for every block of the pair
  const float off[2] = {pg.w[0].off, pg.w[1].off};
  float tx[XV], ku[2][2][XV];
#pragma unroll
  for (int c = 0; c < XV; ++c) {
    const int x = M::col(tid, c);
    const float u = (float)(x - N / 2);
    tx[c] = a.taper[x];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      ku[m][0][c] = wn.ra[m].f11 * u;
      ku[m][1][c] = wn.ra[m].f21 * u;
    }
  }
  float s[6] = {0, 0, 0, 0, 0, 0};
  float s3c[2][XV];
#pragma unroll
  for (int c = 0; c < XV; ++c) s3c[0][c] = s3c[1][c] = 0.0f;
  float lateA[NL][XV], lateB[NL][XV];  // stage rows [FL, R) of each image
  bool clamped = false;

  if constexpr (!FAST) __syncthreads();  // row parameters visible
  // Tiled images first: their tile sits at the end of the stage (when FL <
  // R), so an image gathered straight from memory writes all its rows only
  // after every tile has been consumed.
  if (use0) {
    tile_store<tile_cw<N>()>(tile, bufA, wn.tg[0], wn.im[0], bd0, tid);
    __syncthreads();
    if (tr0)
      gather_rows_trans<N, R, FL, NL, false>(stage, lateA, tile, wn.tg[0], wn.pt[0], a.taper, y0, wn.im[0], bd0, tx,
                                             off[0], tid, s[1], s3c[0], clamped);
    else
      gather_rows<N, R, FL, NL, false, true>(stage, lateA, tile, wn.tg[0], sh.rparam[0], sh.trow, ku[0], wn.im[0],
                                             bd0, tx, off[0], tid, s[1], s3c[0], clamped);
  }
  if (use1) {
    if (use0) __syncthreads();  // tile of A fully consumed
    tile_store<tile_cw<N>()>(tile, bufB, wn.tg[1], wn.im[1], bd1, tid);
    __syncthreads();
    if (tr1)
      gather_rows_trans<N, R, FL, NL, true>(stage, lateB, tile, wn.tg[1], wn.pt[1], a.taper, y0, wn.im[1], bd1, tx,
                                            off[1], tid, s[4], s3c[1], clamped);
    else
      gather_rows<N, R, FL, NL, true, true>(stage, lateB, tile, wn.tg[1], sh.rparam[1], sh.trow, ku[1], wn.im[1],
                                            bd1, tx, off[1], tid, s[4], s3c[1], clamped);
  }
  if constexpr (!FAST) {
    if (FL < R && (use0 || use1) && !(use0 && use1)) __syncthreads();  // tile consumed
    if (!use0)
      gather_rows<N, R, R, NL, false, false>(stage, lateA, tile, wn.tg[0], sh.rparam[0], sh.trow, ku[0], wn.im[0],
                                             true, tx, off[0], tid, s[1], s3c[0], clamped);
    if (!use1)
      gather_rows<N, R, R, NL, true, false>(stage, lateB, tile, wn.tg[1], sh.rparam[1], sh.trow, ku[1], wn.im[1],
                                            true, tx, off[1], tid, s[4], s3c[1], clamped);
  }
#pragma unroll
  for (int c = 0; c < XV; ++c) {
    s[2] = fmaf(tx[c], s3c[0][c], s[2]);
    s[5] = fmaf(tx[c], s3c[1][c], s[5]);
  }
  if constexpr (FL < R) {
    // rows [FL, R) of the tiled images (they overlap the tile)
    if (use0 && use1) __syncthreads();  // tile of B fully consumed
    float* st = reinterpret_cast<float*>(stage);
#pragma unroll
    for (int i = 0; i < R - FL; ++i)
#pragma unroll
      for (int c = 0; c < XV; ++c) {
        const int q = 2 * ((FL + i) * RS + lidx(FwdMap<N, R>::col(tid, c)));
        if (use0) st[q] = lateA[i][c];
        if (use1) st[q + 1] = lateB[i][c];
      }
  }
  __syncthreads();
  if constexpr (PEARSON) {
    pearson_rows<N, R, RS>(stage, a, pair, y0, tid, s);
    __syncthreads();
  }

  // row FFTs in place: transform g of iteration it owns stage row g + it*G
  Twiddles<N> tw;
  tw_load<N>(tw, t, a.tw);
  // the DC bins (lane t = 0 of each transform) sum a'T and b'T over the rows
  float dcA = 0.0f, dcB = 0.0f;
#pragma unroll 1
  for (int it = 0; it < R / G; ++it) {
    float2* row = stage + (g + it * G) * RS;
    float2 d[E];
#pragma unroll
    for (int e = 0; e < E; ++e) d[e] = row[lidx(t + e * T)];
    wave_lds_sync();
    fft_wave<N, false>(d, row, t, tw);
#pragma unroll
    for (int e = 0; e < E; ++e) row[lidx(t + e * T)] = d[e];
    dcA += t == 0 ? d[0].x : 0.0f;
    dcB += t == 0 ? d[0].y : 0.0f;
  }
  if constexpr (!PEARSON) s[0] = dcA;  // (the Pearson template sum comes from pearson_rows)
  s[3] = dcB;

  // slice sums; with one transform per wave only lane 0 holds the DC sums
  const int wv = tid >> 6, ln = tid & 63;
  double acc[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    if (T == 64 && (i == 3 || (i == 0 && !PEARSON)))
      acc[i] = (double)__int_as_float(__builtin_amdgcn_readlane(__float_as_int(s[i]), 0));
    else
      acc[i] = (double)wave_sum_f32(s[i]);
  }
  const int anyc = __any(clamped) ? 1 : 0;
  if (ln == 0) {
#pragma unroll
    for (int i = 0; i < 6; ++i) sh.red[wv][i] = acc[i];
    sh.redc[wv] = anyc;
  }
  __syncthreads();
  if (tid == 0) {
    RowPart rp;
#pragma unroll
    for (int i = 0; i < 6; ++i) rp.s[i] = sh.red[0][i] + sh.red[1][i] + sh.red[2][i] + sh.red[3][i];
    rp.clamped = sh.redc[0] | sh.redc[1] | sh.redc[2] | sh.redc[3];
    rp.off[0] = off[0];
    rp.off[1] = off[1];
    rp.pad = 0;
    a.rowpart[(size_t)pair * NSLICE + slice] = rp;
  }

  // store in the tiled layout: Z[pair][y / 8][kx][y % 8].  A thread writes
  // the float4 of rows (r, r + 1) at bin kx; with R >= 8 the block's region is
  // contiguous and consecutive threads write consecutive 16-byte chunks.  The
  // thread's chunk of round i is a constant distance from that of round 0
  // (in the stage and in Z), so the rounds differ by immediate offsets.
  {
    constexpr int Q = N * R / 2;
    static_assert(Q % 256 == 0 && (R >= 8 || 8 % R == 0), "store rounds");
    // round 0: kx0 = thread's bin, r0 its first row (of a pair)
    constexpr int RP = R >= 8 ? 4 : R / 2;  // row pairs per column in one round
    const int kx0 = tid / RP, r0 = 2 * (tid % RP);
    float4* zb = reinterpret_cast<float4*>(a.Z + (size_t)pair * N * N) +
                 (ztile<N>(kx0, (y0 & ~7) + ((R >= 8 ? 0 : y0 & 7) + r0)) >> 1);
    const float2* sb = stage + r0 * RS + lidx(kx0);
#pragma unroll
    for (int i = 0; i < Q / 256; ++i) {
      // round i adds dq = 256 i to the chunk index q = (y / 8) 4N + kx RP + (r / 2) (R >= 8)
      // or q = kx RP + r / 2 (R < 8)
      const int dq = 256 * i;
      const int dyt = R >= 8 ? dq / (4 * N) : 0;        // whole 8-row tiles
      const int dkx = (R >= 8 ? dq % (4 * N) : dq) / RP;  // a multiple of 64
      // lidx(kx0 + dkx) = lidx(kx0) + lidx(dkx) for dkx a multiple of 32
      const float2 v0 = sb[dyt * 8 * RS + lidx(dkx)], v1 = sb[(dyt * 8 + 1) * RS + lidx(dkx)];
      zb[(dyt * 8 * N + dkx * 8) >> 1] = make_float4(v0.x, v0.y, v1.x, v1.y);
    }
  }
}

template <int N, int R, int BUDGET, int TRW, bool PEARSON>
__global__ void __launch_bounds__(256) k_row_fwd(MatchArgs a) {
  using C = FftCfg<N>;
  constexpr int T = C::T, G = 256 / T, NSLICE = N / R;
  static_assert(R % G == 0 && (N * R) % 256 == 0 && 2 * R <= 64, "row split");
  __shared__ FwdLds<N, R, BUDGET> sh;

  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int pair = blk / NSLICE, slice = blk % NSLICE, y0 = slice * R;
  const int tid = threadIdx.x;

  // image indices are clamped into the table so a bad index cannot read past it
  const int ka = min(max(a.img_a[pair], 0), a.n_imgs - 1);
  const int kb = min(max(a.img_b[pair], 0), a.n_imgs - 1);
  FwdWin wn;
  wn.im[0] = a.imgs[ka];
  wn.im[1] = a.imgs[kb];
  const float* th[2] = {a.th_a + 8 * (size_t)pair, a.th_b + 8 * (size_t)pair};
  const PairGeom pg = a.geom[pair];  // origin split, translation test, offsets (k_pair_geom)
  using M = FwdMap<N, R>;
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    wn.im[m].width = max(wn.im[m].width, 2);
    wn.im[m].height = max(wn.im[m].height, 2);
    // translation windows (identity linear part) take the constant-weight
    // gather, and their tile geometry and row parameters are integer offsets
    // from floor(cx + tx), floor(cy + ty); only other windows need the affine
    wn.trans[m] = (pg.w[m].flags & 1) != 0;
    if (wn.trans[m]) {
      const int bx0 = pg.w[m].bx0, by0 = pg.w[m].by0;
      wn.tg[m] = tile_geom_trans<N, R, BUDGET, TRW>(bx0, by0, (pg.w[m].flags & 2) != 0, wn.im[m], y0);
      wn.pt[m].bx = bx0 - (wn.tg[m].use ? wn.tg[m].xlo : 0);
      wn.pt[m].by = by0 + (y0 + M::row0(tid) - N / 2) - (wn.tg[m].use ? wn.tg[m].ylo : 0);
      wn.pt[m].fx = pg.w[m].fx;
      wn.pt[m].fy = pg.w[m].fy;
      wn.ra[m].xc = wn.ra[m].yc = 0.0;
      wn.ra[m].a11 = wn.ra[m].a22 = 1.0;
      wn.ra[m].a12 = wn.ra[m].a21 = 0.0;
      wn.ra[m].f11 = 1.0f;
      wn.ra[m].f21 = 0.0f;
    } else {
      wn.ra[m] = row_affine(th[m]);
      wn.tg[m] = tile_geom<N, R, BUDGET, TRW>(wn.ra[m], wn.im[m], y0);
      wn.pt[m].bx = wn.pt[m].by = 0;
      wn.pt[m].fx = wn.pt[m].fy = 0.0f;
    }
    // could any sample read outside the image?  (one pixel of slack for rounding)
    const TileGeom& tg = wn.tg[m];
    wn.border[m] = !(tg.use && tg.xlo >= 0 && tg.xlo + 4 * tg.wt4 <= wn.im[m].width && tg.ylo >= 0 &&
                     tg.ylo + tg.ht <= wn.im[m].height);
  }
  const bool fast = wn.trans[0] && wn.trans[1] && wn.tg[0].use && wn.tg[1].use && !wn.border[0] && !wn.border[1];
  if (fast)
    row_fwd_body<N, R, BUDGET, TRW, PEARSON, true>(a, sh, wn, pg, pair, slice, y0, tid);
  else
    row_fwd_body<N, R, BUDGET, TRW, PEARSON, false>(a, sh, wn, pg, pair, slice, y0, tid);
}

// ---------------------------------------------------------------- pair statistics
template <int N>
__global__ void __launch_bounds__(64) k_pair_stats(MatchArgs a) {
  const int NSLICE = a.nsl_fwd;
  const int pair = blockIdx.x, ln = threadIdx.x;
  double s[6] = {0, 0, 0, 0, 0, 0};
  int cl = 0;
  for (int i = ln; i < NSLICE; i += 64) {
    const RowPart rp = a.rowpart[(size_t)pair * NSLICE + i];
#pragma unroll
    for (int q = 0; q < 6; ++q) s[q] += rp.s[q];
    cl |= rp.clamped;
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) s[q] = wave_sum(s[q]);
  cl = __any(cl) ? 1 : 0;
  if (ln == 0) {
    const RowPart r0 = a.rowpart[(size_t)pair * NSLICE];
    const PairStat ps = make_pair_stat(s, cl != 0, *a.tinfo, r0.off[0], r0.off[1], N, a.pearson != 0, a.p);
    a.pstat[pair] = ps;
    if (a.saved_ps) a.saved_ps[pair] = ps;
  }
}

// Sum over the T lanes of one FFT group (groups are aligned runs of T lanes;
// a group is either wholly active or wholly exited).
template <int T>
__device__ __forceinline__ float group_sum_f32(float v) {
  if constexpr (T == 64) {
    return wave_sum_f32(v);
  } else {
#pragma unroll
    for (int off = T / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
  }
}

// Pruned inverse: the column sum of |C|^2 over ky for column kx (weight 2 for
// the columns that stand for their mirror N - kx too), and the stored rows.
template <int N, int T>
__device__ __forceinline__ void col_sumsq(const MatchArgs& a, int pair, int w, int t, float csq) {
  const float tot = group_sum_f32<T>(csq);
  if (t == 0) a.colsq[(size_t)pair * (N / 2 + 1) + w] = (double)tot * ((w == 0 || w == N / 2) ? 1.0 : 2.0);
}

// Column w of the inverse column transform, back into the tiled layout (with
// a search radius only the rows the inverse row blocks read).
template <int N, int T, int E, bool PRUNE>
__device__ __forceinline__ void store_column(const MatchArgs& a, float2* Zp, int w, int t, const float2 (&v)[E]) {
  if (!PRUNE || a.zlo >= N) {
#pragma unroll
    for (int e = 0; e < E; ++e) Zp[ztile<N>(w, t + e * T)] = v[e];
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int y = t + e * T;
      if (y < a.zlo || y >= a.zhi) Zp[ztile<N>(w, y)] = v[e];
    }
  }
}

// ---------------------------------------------------------------- column pass + whitening
// Column pass with one FFT group per column pair: the group transforms
// columns N - kx and kx, splits, whitens and inverse-transforms column kx,
// exchanging the mirror column through its own LDS slot (no block barrier,
// no idle groups).  At 1024^2 (16 elements per lane, two columns in flight)
// the register budget is held to 168 VGPRs, three workgroups per CU, which
// the LDS slots allow.
template <int N, bool PRUNE>
__global__ void __launch_bounds__(256, N >= 1024 ? 3 : 1) k_col_pair(MatchArgs a) {
  using C = FftCfg<N>;
  constexpr int T = C::T, E = C::E, G = 256 / T;
  constexpr int NI = N / 2 + 1, NW = (NI + G - 1) / G;
  constexpr int SL = fft_scratch<N>();
  __shared__ float2 lds[G * SL];

  const int pair = blockIdx.x / NW, wg = blockIdx.x % NW;
  const int tid = threadIdx.x, c = tid / T, t = tid % T;
  const int w = wg * G + c;
  if (w >= NI) return;  // whole groups only; no block-level barrier follows
  const int wm = (N - w) & (N - 1);  // mirror column
  float2* Zp = a.Z + (size_t)pair * N * N;
  float2* slot = lds + c * SL;
  Twiddles<N> tw;
  tw_load<N>(tw, t, a.tw);

  float2 v[E], u[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = Zp[ztile<N>(w, t + e * T)];
  fft_wave<N, false>(v, slot, t, tw);
  wave_lds_sync();
  if (wm != w) {
    // the mirror column is loaded only now, so it is not live during the
    // first transform
#pragma unroll
    for (int e = 0; e < E; ++e) u[e] = Zp[ztile<N>(wm, t + e * T)];
    fft_wave<N, false>(u, slot, t, tw);
    wave_lds_sync();
  } else {
#pragma unroll
    for (int e = 0; e < E; ++e) u[e] = v[e];
  }
  if (a.saved_Z) {
    float2* sz = a.saved_Z + (size_t)pair * N * N;
#pragma unroll
    for (int e = 0; e < E; ++e) sz[(size_t)w * N + t + e * T] = v[e];
    if (wm != w) {
#pragma unroll
      for (int e = 0; e < E; ++e) sz[(size_t)wm * N + t + e * T] = u[e];
    }
  }
#pragma unroll
  for (int e = 0; e < E; ++e) slot[lidx(t + e * T)] = u[e];
  wave_lds_sync();

  const PairStat ps = a.pstat[pair];
  const float2 tauw = a.tau[w];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int ky = t + e * T;
    v[e] = whiten_bin(v[e], cconj(slot[lidx((N - ky) & (N - 1))]), cmul(a.tau[ky], tauw), ps, a.p, a.eps_rel,
                      ky == 0 && w == 0);
  }
  if constexpr (PRUNE) {
    float csq = 0.0f;
#pragma unroll
    for (int e = 0; e < E; ++e) csq = fmaf(v[e].x, v[e].x, fmaf(v[e].y, v[e].y, csq));
    col_sumsq<N, T>(a, pair, w, t, csq);
  }
  wave_lds_sync();  // every lane has read its mirror values
  fft_wave<N, true>(v, slot, t, tw);
  store_column<N, T, E, PRUNE>(a, Zp, w, t, v);
}

// ---------------------------------------------------------------- Pearson patch energies
// Column half of the cumulative-area correction: for placement (i, j) =
// (sy + N/4, sx + N/4) the patch covers rows [i, i + N/2) of the row sums of
// column j, so a running FP64 window down the rows gives E1 = sum f', E2 =
// sum f'^2 and the energy E2 - E1^2 / m^2 (m^2 patch pixels).  One thread per
// placement column j.
template <int N>
__global__ void __launch_bounds__(64) k_ncc_energy(MatchArgs a) {
  constexpr int M = N / 2, NP = N / 2 + 1, NB = (NP + 63) / 64;
  const int pair = blockIdx.x / NB, j = (blockIdx.x % NB) * 64 + threadIdx.x;
  if (j >= NP) return;
  const float2* rb = a.ncc_rows + (size_t)pair * N * NP + j;
  float* V = a.ncc_var + (size_t)pair * NP * NP + j;
  constexpr int U = 8;  // rows per batch of loads, all issued before any store
  static_assert(M % U == 0, "placements per column minus one divide into batches");
  double e1 = 0.0, e2 = 0.0;
  for (int y0 = 0; y0 < M; y0 += U) {
    float2 r[U];
#pragma unroll
    for (int u = 0; u < U; ++u) r[u] = rb[(size_t)(y0 + u) * NP];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      e1 += r[u].x;
      e2 += r[u].y;
    }
  }
  const double inv = 1.0 / ((double)M * (double)M);
  V[0] = (float)fmax(e2 - e1 * e1 * inv, 0.0);
  for (int i0 = 1; i0 < NP; i0 += U) {
    float2 ro[U], rn[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ro[u] = rb[(size_t)(i0 + u - 1) * NP];
      rn[u] = rb[(size_t)(i0 + u + M - 1) * NP];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      e1 += (double)rn[u].x - (double)ro[u].x;
      e2 += (double)rn[u].y - (double)ro[u].y;
      V[(size_t)(i0 + u) * NP] = (float)fmax(e2 - e1 * e1 * inv, 0.0);
    }
  }
}

// Pearson coefficient of placement (sy, sx) from the correlation value c, the
// template energy st and the patch energy; 0 when either energy is 0.
template <int N>
__device__ __forceinline__ float pearson_gamma(const MatchArgs& a, int pair, int sy, int sx, float c, float st) {
  constexpr int NP = N / 2 + 1;
  const float v = a.ncc_var[((size_t)pair * NP + (sy + N / 4)) * NP + (sx + N / 4)];
  const float den = st * v;
  return den > 0.0f ? c * rsqrtf(den) : 0.0f;
}

// ---------------------------------------------------------------- row pass (inverse) + statistics
// PRUNE: the launched row blocks are the first a.nsl_lo and the last
// a.nsl_inv - a.nsl_lo of the N / R2 blocks of a pair; the peak is searched
// among wrapped shifts |sx|, |sy| <= a.max_shift; no sums (the background
// comes from the spectrum).
// PEARSON (with PRUNE, radius N/4): the candidates are the Pearson
// coefficients of the placements, and the sums are over those coefficients.
template <int N, int R2, bool PRUNE, bool PEARSON>
__global__ void __launch_bounds__(256) k_row_inv(MatchArgs a) {
  static_assert(PRUNE || !PEARSON, "the Pearson search runs on the pruned rows");
  using C = FftCfg<N>;
  constexpr int T = C::T, E = C::E, G = 256 / T, NT = R2 / 2, NSL2 = N / R2;
  // a row pair holds a transform's scratch; the stage load (thread row
  // tid % R2) hits distinct banks
  constexpr int NH = N / 2 + 1, RS2 = rows_stride<R2>((fft_scratch<N>() + 1) / 2 > NH ? (fft_scratch<N>() + 1) / 2 : NH);
  static_assert(2 * RS2 >= fft_scratch<N>(), "row pair must hold the FFT scratch");
  __shared__ float2 stage[R2 * RS2];
  __shared__ float rm1[4], rm2[4];
  __shared__ int ri1[4];
  __shared__ double rs[4], rq[4];

  const int NSP = PRUNE ? a.nsl_inv : NSL2;
  const int pair = blockIdx.x / NSP, sl = blockIdx.x % NSP;
  const int slice = (!PRUNE || sl < a.nsl_lo) ? sl : NSL2 - (NSP - sl);
  const int y0 = slice * R2;
  const int rmax = PRUNE ? a.max_shift : 0;
  const float st = PEARSON ? a.pstat[pair].swA : 0.0f;
  const int tid = threadIdx.x, g = tid / T, t = tid % T;
  const float2* Zp = a.Z + (size_t)pair * N * N;

  {
    // thread: row r = tid % R2 of columns c0 + k CPL.  Only the last round
    // can pass column N/2 (ceil(NH / CPL) rounds); its column is clamped so
    // every load stays in bounds and all of them are in flight at once.
    static_assert(256 % R2 == 0, "rows per block divide the block");
    constexpr int CPL = 256 / R2, LD = (NH + CPL - 1) / CPL;
    const int r = tid % R2, c0 = tid / R2;
    // tiled layout: column c of row y at ztile(c, y), so the k-th load is a
    // constant 8 CPL elements past the first
    const char* zb = reinterpret_cast<const char*>(Zp);
    const uint32_t off0 = (uint32_t)ztile<N>(c0, y0 + r) * (uint32_t)sizeof(float2);
    float2 buf[LD];
#pragma unroll
    for (int k = 0; k < LD - 1; ++k)
      buf[k] = *reinterpret_cast<const float2*>(zb + off0 + (uint32_t)(k * CPL * 8 * sizeof(float2)));
    {
      const int cl = min(c0 + (LD - 1) * CPL, NH - 1);
      buf[LD - 1] = Zp[ztile<N>(cl, y0 + r)];
    }
    float2* sp = stage + r * RS2 + c0;
#pragma unroll
    for (int k = 0; k < LD - 1; ++k) sp[k * CPL] = buf[k];
    if (c0 + (LD - 1) * CPL < NH) sp[(LD - 1) * CPL] = buf[LD - 1];
  }
  __syncthreads();

  Top2 tp;
  tp.m1 = -FLT_MAX;
  tp.i1 = INT_MAX;
  tp.m2 = -FLT_MAX;
  double sum = 0.0, sq = 0.0;
  float* surf = a.surfaces ? a.surfaces + (size_t)pair * N * N : nullptr;
  Twiddles<N> tw;
  tw_load<N>(tw, t, a.tw);

#pragma unroll 1
  for (int it = 0; it < (NT + G - 1) / G; ++it) {
    const int c = g + it * G;
    if (c < NT) {
      float2* r1 = stage + (2 * c) * RS2;
      float2* r2 = r1 + RS2;
      float2 v[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int k = t + e * T;
        float2 g1, g2;
        if (k <= N / 2) {
          g1 = r1[k];
          g2 = r2[k];
        } else {
          g1 = cconj(r1[N - k]);
          g2 = cconj(r2[N - k]);
        }
        v[e] = make_float2(g1.x - g2.y, g1.y + g2.x);
      }
      wave_lds_sync();
      fft_wave<N, true>(v, r1, t, tw);
      // each lane visits its flat indices in increasing order (row ya, then
      // row yb; rows grow with the iteration), so a strict > keeps the first maximum
      const int ya = y0 + 2 * c, yb = ya + 1;
      if constexpr (PEARSON) {
        const bool ina = ya <= rmax || ya >= N - rmax, inb = yb <= rmax || yb >= N - rmax;
        const int sya = ya >= N / 2 ? ya - N : ya, syb = yb >= N / 2 ? yb - N : yb;
        float ls = 0.0f, lq = 0.0f;
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const int x = t + e * T;
          if (ina && (x <= rmax || x >= N - rmax)) {
            const float gv = pearson_gamma<N>(a, pair, sya, x >= N / 2 ? x - N : x, v[e].x, st);
            top2_push_ordered(tp, gv, ya * N + x);
            ls += gv;
            lq = fmaf(gv, gv, lq);
          }
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const int x = t + e * T;
          if (inb && (x <= rmax || x >= N - rmax)) {
            const float gv = pearson_gamma<N>(a, pair, syb, x >= N / 2 ? x - N : x, v[e].y, st);
            top2_push_ordered(tp, gv, yb * N + x);
            ls += gv;
            lq = fmaf(gv, gv, lq);
          }
        }
        sum += (double)ls;
        sq += (double)lq;
        continue;
      } else if constexpr (PRUNE) {
        const bool ina = ya <= rmax || ya >= N - rmax, inb = yb <= rmax || yb >= N - rmax;
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const int x = t + e * T;
          if (ina && (x <= rmax || x >= N - rmax)) top2_push_ordered(tp, v[e].x, ya * N + x);
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const int x = t + e * T;
          if (inb && (x <= rmax || x >= N - rmax)) top2_push_ordered(tp, v[e].y, yb * N + x);
        }
        continue;
      }
      float ls = 0.0f, lq = 0.0f;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const float ca = v[e].x;
        top2_push_ordered(tp, ca, ya * N + t + e * T);
        ls += ca;
        lq = fmaf(ca, ca, lq);
      }
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const float cb = v[e].y;
        top2_push_ordered(tp, cb, yb * N + t + e * T);
        ls += cb;
        lq = fmaf(cb, cb, lq);
      }
      sum += (double)ls;
      sq += (double)lq;
      if (surf) {
#pragma unroll
        for (int e = 0; e < E; ++e) {
          surf[(size_t)ya * N + t + e * T] = v[e].x;
          surf[(size_t)yb * N + t + e * T] = v[e].y;
        }
      }
    }
  }
  tp = wave_top2(tp);
  sum = wave_sum(sum);
  sq = wave_sum(sq);
  const int wv = tid >> 6, ln = tid & 63;
  if (ln == 0) {
    rm1[wv] = tp.m1;
    ri1[wv] = tp.i1;
    rm2[wv] = tp.m2;
    rs[wv] = sum;
    rq[wv] = sq;
  }
  __syncthreads();
  if (tid == 0) {
    Top2 b;
    b.m1 = rm1[0];
    b.i1 = ri1[0];
    b.m2 = rm2[0];
    for (int i = 1; i < 4; ++i) {
      Top2 o;
      o.m1 = rm1[i];
      o.i1 = ri1[i];
      o.m2 = rm2[i];
      b = top2_merge(b, o);
    }
    InvPart ip;
    ip.m1 = b.m1;
    ip.i1 = b.i1;
    ip.m2 = b.m2;
    ip.pad = 0;
    ip.sum = rs[0] + rs[1] + rs[2] + rs[3];
    ip.sumsq = rq[0] + rq[1] + rq[2] + rq[3];
    a.invpart[(size_t)pair * NSP + sl] = ip;
  }
}

// ---------------------------------------------------------------- finalize
template <int N>
__global__ void __launch_bounds__(64) k_finalize(MatchArgs a) {
  using C = FftCfg<N>;
  constexpr int T = C::T, E = C::E;
  const int NSL2 = a.nsl_inv;
  constexpr int SL = fft_scratch<N>();
  __shared__ float2 lds[SL];
  __shared__ float nb[3][3];
  const int pair = blockIdx.x, ln = threadIdx.x;

  Top2 tp;
  tp.m1 = -FLT_MAX;
  tp.i1 = INT_MAX;
  tp.m2 = -FLT_MAX;
  double sum = 0.0, sq = 0.0;
  for (int i = ln; i < NSL2; i += 64) {
    const InvPart ip = a.invpart[(size_t)pair * NSL2 + i];
    Top2 o;
    o.m1 = ip.m1;
    o.i1 = ip.i1;
    o.m2 = ip.m2;
    tp = top2_merge(tp, o);
    sum += ip.sum;
    sq += ip.sumsq;
  }
  tp = wave_top2(tp);
  sum = wave_sum(sum);
  sq = wave_sum(sq);
  if (a.max_shift > 0 && !a.pearson) {
    // pruned: sum_x c = C(0) = 0, and by Parseval sum_x c^2 = N^2 sum_k |C(k)|^2
    // (C here carries the inverse transform's 1/N^2)
    double cs = 0.0;
    for (int i = ln; i < N / 2 + 1; i += 64) cs += a.colsq[(size_t)pair * (N / 2 + 1) + i];
    cs = wave_sum(cs);
    sum = 0.0;
    sq = (double)N * (double)N * cs;
  }
  const int flat = (tp.i1 >= 0 && tp.i1 < N * N) ? tp.i1 : 0;
  const int iy = flat / N, ix = flat % N;
  const float2* Zp = a.Z + (size_t)pair * N * N;

  // recompute the surface rows iy - RB .. iy + RB, two per complex FFT: the
  // 3 x 3 neighbourhood of the peak, and with snr_exclude_r = R > 0 the sums
  // over the (2R+1)^2 box the background leaves out
  const int R = a.pearson ? 0 : a.snr_exclude_r, RB = R > 1 ? R : 1;
  double bs = 0.0, bq = 0.0;
  for (int r0 = -RB; r0 <= RB; r0 += 2) {
    const int ra = (iy + r0) & (N - 1);
    const bool two = r0 + 1 <= RB;
    const int rb = two ? ((iy + r0 + 1) & (N - 1)) : -1;
    if (ln < T) {
      float2 v[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int k = ln + e * T;
        const int kk = k <= N / 2 ? k : N - k;
        float2 g1 = Zp[ztile<N>(kk, ra)];
        float2 g2 = rb >= 0 ? Zp[ztile<N>(kk, rb)] : make_float2(0.f, 0.f);
        if (k > N / 2) {
          g1 = cconj(g1);
          g2 = cconj(g2);
        }
        v[e] = make_float2(g1.x - g2.y, g1.y + g2.x);
      }
      fft_wave_tab<N, true>(v, lds, ln, a.tw);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int x = ln + e * T;
        int dxi = x - ix;
        if (dxi > N / 2) dxi -= N;
        if (dxi < -N / 2) dxi += N;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int dy = r0 + h;
          if (h == 1 && !two) continue;
          const float cv = h == 0 ? v[e].x : v[e].y;
          if (dxi >= -1 && dxi <= 1 && dy >= -1 && dy <= 1) nb[dy + 1][dxi + 1] = cv;
          if (dxi >= -R && dxi <= R && dy >= -R && dy <= R) {
            // the peak itself enters with the value the search found
            const double c = (dxi == 0 && dy == 0) ? (double)tp.m1 : (double)cv;
            bs += c;
            bq += c * c;
          }
        }
      }
    }
    __syncthreads();
  }
  bs = wave_sum(bs);
  bq = wave_sum(bq);

  if (ln == 0) {
    const PairStat ps = a.pstat[pair];
    double count = 0.0;
    bool outside = false;
    if (a.pearson) {
      // neighbours as Pearson coefficients; placements beyond the search range
      // get the lowest value, so they weigh nothing in the centroid
      constexpr int RP = N / 4;
      const int sy0 = iy >= N / 2 ? iy - N : iy, sx0 = ix >= N / 2 ? ix - N : ix;
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const int sy = sy0 + dy, sx = sx0 + dx;
          if (sy < -RP || sy > RP || sx < -RP || sx > RP) {
            nb[dy + 1][dx + 1] = -FLT_MAX;
            outside = true;
          } else {
            nb[dy + 1][dx + 1] = pearson_gamma<N>(a, pair, sy, sx, nb[dy + 1][dx + 1], ps.swA);
          }
        }
      count = (double)(2 * RP + 1) * (double)(2 * RP + 1);
    }
    if (R > 0) {
      // background without the box: M - (2R+1)^2 entries
      sum -= bs;
      sq -= bq;
      count = (double)N * (double)N - (double)(2 * R + 1) * (double)(2 * R + 1);
    }
    swift_match rec = make_record(N, tp, sum, sq, nb, (ps.flags & 4) ? SWIFT_ST_CLAMPED : 0, count);
    if (outside) rec.hxx = rec.hyy = rec.hxy = 0.0f;
    a.out[pair] = rec;
    if (a.saved_rec) a.saved_rec[pair] = rec;
    if (a.saved_nb)
      for (int q = 0; q < 9; ++q) a.saved_nb[(size_t)pair * 9 + q] = nb[q / 3][q % 3];
  }
}

// ---------------------------------------------------------------- launchers
size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

hipError_t launch_taper(int n, float taper_frac, float2* tau, float* taper, TaperInfo* info, hipStream_t s,
                        bool box) {
  if (box) {
    k_taper_box<<<(n + 255) / 256, 256, 0, s>>>(n, tau, taper, info);
    return hipGetLastError();
  }
  const int L = (int)floor((double)taper_frac * n / 2.0 + 0.5);
  k_taper<<<(n + 255) / 256, 256, 0, s>>>(n, L, tau, taper, info);
  return hipGetLastError();
}

struct TimerScope {
  KernelTimer* kt;
  hipStream_t s;
  TimerScope(KernelTimer* k, const char* name, int n, hipStream_t st) : kt(k), s(st) {
    if (kt) kt->begin(name, n, s);
  }
  ~TimerScope() {
    if (kt) kt->end(s);
  }
};

template <int N, int R, int BUDGET, int TRW, int R2>
static hipError_t launch_group_v(const MatchArgs& a, hipStream_t s, KernelTimer* kt) {
  using C = FftCfg<N>;
  constexpr int G = 256 / C::T;
  const unsigned P = (unsigned)a.npairs;
  if (a.nsl_fwd != N / R) return hipErrorInvalidValue;
  if (a.max_shift > 0 ? (a.nsl_inv > N / R2 || a.nsl_lo > a.nsl_inv) : (a.nsl_inv != N / R2))
    return hipErrorInvalidValue;
  if (a.pearson && a.max_shift != N / 4) return hipErrorInvalidValue;
  {
    TimerScope ts(kt, "k_pair_geom", N, s);
    k_pair_geom<<<(P + 255) / 256, 256, 0, s>>>(a);
  }
  {
    TimerScope ts(kt, "k_row_fwd", N, s);
    if (a.pearson)
      k_row_fwd<N, R, BUDGET, TRW, true><<<P * (N / R), 256, 0, s>>>(a);
    else
      k_row_fwd<N, R, BUDGET, TRW, false><<<P * (N / R), 256, 0, s>>>(a);
  }
  {
    TimerScope ts(kt, "k_pair_stats", N, s);
    k_pair_stats<N><<<P, 64, 0, s>>>(a);
  }
  if (a.pearson) {
    TimerScope ts(kt, "k_ncc_energy", N, s);
    constexpr int NB = (N / 2 + 1 + 63) / 64;
    k_ncc_energy<N><<<P * NB, 64, 0, s>>>(a);
  }
  {
    TimerScope ts(kt, "k_col", N, s);
    constexpr int NW2 = (N / 2 + 1 + G - 1) / G;
    if (a.max_shift > 0)
      k_col_pair<N, true><<<P * NW2, 256, 0, s>>>(a);
    else
      k_col_pair<N, false><<<P * NW2, 256, 0, s>>>(a);
  }
  {
    TimerScope ts(kt, "k_row_inv", N, s);
    if (a.pearson)
      k_row_inv<N, R2, true, true><<<P * (unsigned)a.nsl_inv, 256, 0, s>>>(a);
    else if (a.max_shift > 0)
      k_row_inv<N, R2, true, false><<<P * (unsigned)a.nsl_inv, 256, 0, s>>>(a);
    else
      k_row_inv<N, R2, false, false><<<P * (N / R2), 256, 0, s>>>(a);
  }
  {
    TimerScope ts(kt, "k_finalize", N, s);
    k_finalize<N><<<P, 64, 0, s>>>(a);
  }
  return hipGetLastError();
}

template <int N>
static hipError_t launch_group_t(const MatchArgs& a, bool alt_fwd, bool alt_inv, hipStream_t s, KernelTimer* kt) {
  using RC = RowsCfg<N>;
  if (!alt_fwd && !alt_inv) return launch_group_v<N, RC::FWD, RC::TILE, RC::TRW, RC::INV>(a, s, kt);
  if (!alt_fwd && alt_inv) return launch_group_v<N, RC::FWD, RC::TILE, RC::TRW, RC::INV2>(a, s, kt);
  if (alt_fwd && !alt_inv) return launch_group_v<N, RC::FWD2, RC::TILE2, RC::TRW2, RC::INV>(a, s, kt);
  return launch_group_v<N, RC::FWD2, RC::TILE2, RC::TRW2, RC::INV2>(a, s, kt);
}

int fwd_blocks_n(int n, bool alt) {
  switch (n) {
    case 64: return 64 / (alt ? RowsCfg<64>::FWD2 : RowsCfg<64>::FWD);
    case 128: return 128 / (alt ? RowsCfg<128>::FWD2 : RowsCfg<128>::FWD);
    case 256: return 256 / (alt ? RowsCfg<256>::FWD2 : RowsCfg<256>::FWD);
    case 512: return 512 / (alt ? RowsCfg<512>::FWD2 : RowsCfg<512>::FWD);
    default: return 1024 / (alt ? RowsCfg<1024>::FWD2 : RowsCfg<1024>::FWD);
  }
}

int inv_blocks_n(int n, bool alt) {
  switch (n) {
    case 64: return 64 / (alt ? RowsCfg<64>::INV2 : RowsCfg<64>::INV);
    case 128: return 128 / (alt ? RowsCfg<128>::INV2 : RowsCfg<128>::INV);
    case 256: return 256 / (alt ? RowsCfg<256>::INV2 : RowsCfg<256>::INV);
    case 512: return 512 / (alt ? RowsCfg<512>::INV2 : RowsCfg<512>::INV);
    default: return 1024 / (alt ? RowsCfg<1024>::INV2 : RowsCfg<1024>::INV);
  }
}

hipError_t launch_match_group(int n, const MatchArgs& a, int fwd_variant, bool alt_inv, hipStream_t s, KernelTimer* kt) {
  if (fwd_variant == kFusedVariant && n <= kFusedMaxN && !a.pearson) return launch_fused_group(n, a, s, kt);
  const bool alt_fwd = fwd_variant == 1;
  switch (n) {
    case 64: return launch_group_t<64>(a, alt_fwd, alt_inv, s, kt);
    case 128: return launch_group_t<128>(a, alt_fwd, alt_inv, s, kt);
    case 256: return launch_group_t<256>(a, alt_fwd, alt_inv, s, kt);
    case 512: return launch_group_t<512>(a, alt_fwd, alt_inv, s, kt);
    case 1024: return launch_group_t<1024>(a, alt_fwd, alt_inv, s, kt);
  }
  return hipErrorInvalidValue;
}

}  // namespace swift
