// Whitened FFT window matching for small windows (N = 64, 128): the whole
// pair in one workgroup.
//
// Same method and results as the five-kernel path (Wetzel et al., arXiv
// 1612.04787, Section III: taper, Fourier transforms, amplitudes raised to the
// power p, inverse transform, Z-score of the peak), but the packed field
// z = a'T + i b'T of a pair (N x N complex values, 136 KB at N = 128) stays in
// LDS from the gather to the record, so only the two uint8 windows and the
// 64-byte record cross HBM.  At these sizes the transforms are short and the
// work per byte is high, so the path is bound by the vector ALUs, not by HBM.
//
// Phases, separated by workgroup barriers:
//   1. gather both windows (bilinear affine samples about the centre pixel,
//      taper), window sums;
//   2. row FFTs of z in place (each FFT group of T lanes owns a row);
//   3. pair statistics (weighted means, energies, whitening scales);
//   4. column FFTs of columns kx and N - kx, split into F_A, F_B, whitening,
//      inverse column FFT of column kx (kx <= N/2), in place;
//   5. inverse row FFTs, two real surface rows per complex FFT; top-2 search
//      and FP64 surface sums; the surface stays in LDS;
//   6. record: peak, Z-score (background without the (2R+1)^2 box when asked),
//      3 x 3 centroid read from the LDS surface.
#include <float.h>
#include <limits.h>
#include <math.h>

#include "swift_dev.hpp"
#include "swift_tile.hpp"

namespace swift {

// NTH threads per workgroup, one FFT group per column pair (G = NTH / T =
// N / 2).  S: LDS row stride of z in complex values, at least lidx(N) (a row
// is its own FFT scratch) and chosen so that the T consecutive rows a column
// FFT group reads fall on distinct LDS banks: 2 S mod 64 is 8 (N = 64, T = 8)
// or 20 (N = 128, T = 16).  Source tiles: TB bytes per image at most, fetched
// with TRW 16-byte loads per thread.  During the gather z's storage holds
// window A's samples (N^2 floats) followed by the two tiles; z itself is
// written once both windows are gathered.
template <int N> struct FusedCfg;
template <> struct FusedCfg<64>  { static constexpr int NTH = 256,  S = 68,  TRW = 3, TB = 9200; };
template <> struct FusedCfg<128> { static constexpr int NTH = 1024, S = 138, TRW = 3, TB = 36864; };

// One window's samples for the thread's column x and rows r0 .. r0 + IT - 1,
// at = ((sample - o) t(x)) t(y), with sum at^2 (s2) and sum_r at t(r) (s3);
// ORs the clamp flag into cl.  From the window's LDS tile: a translation
// window takes one horizontal interpolation per tile row (reused by the next
// output row), any other window the bilinear sample of each pixel.
template <int N, int IT>
__device__ __forceinline__ void gather_tile(float (&at)[IT], const uint32_t* __restrict__ tile, const TileGeom& g,
                                            bool trans, const RowParam& p0, const RowParam* __restrict__ rp,
                                            const float* __restrict__ taper_s, const swift_image& im, bool border,
                                            float kux, float kuy, float o, float tx, int x, int r0, float& s2,
                                            float& s3, bool& cl) {
  s2 = 0.0f;
  s3 = 0.0f;
  if (trans) {
    // bytes ix, ix + 1 of tile rows p0.by .. p0.by + IT (the tile keeps a
    // pixel of margin on every side, so no clamping)
    const int ix = p0.bx + (x - N / 2);
    if (border)
      cl |= (ix + g.xlo < 0) | (ix + g.xlo > im.width - 2) | (p0.by + g.ylo < 0) |
            (p0.by + IT - 1 + g.ylo > im.height - 2);
    const uint32_t* wb = tile + p0.by * g.ts + (ix >> 2);
    const uint32_t sh = (uint32_t)(ix & 3);
    const float fx = p0.fx, fy = p0.fy;
    auto hrow = [&](int i) {
      const uint32_t* w = wb + i * g.ts;
      const uint32_t v = __builtin_amdgcn_alignbyte(w[1], w[0], sh);
      const float b0 = (float)(v & 255u), b1 = (float)((v >> 8) & 255u);
      return fmaf(fx, b1 - b0, b0 - o);
    };
    float h0 = hrow(0);
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const float h1 = hrow(i + 1);
      const float val = fmaf(fy, h1 - h0, h0);  // sample - o
      h0 = h1;
      const float ty = taper_s[r0 + i];
      const float a = (val * tx) * ty;
      s2 = fmaf(a, a, s2);
      s3 = fmaf(a, ty, s3);
      at[i] = a;
    }
    return;
  }
  const int rowb = g.ts * 4;
#pragma unroll
  for (int i = 0; i < IT; ++i) {
    const int r = r0 + i;
    const RowParam p = rp[r];
    const float ty = taper_s[r];
    const float xr = p.fx + kux, yr = p.fy + kuy;
    const float xf = floorf(xr), yf = floorf(yr);
    const float fx = xr - xf, fy = yr - yf;
    const int x0 = p.bx + (int)xf, y0 = p.by + (int)yf;
    // branch-free, so the rows stay one block the scheduler can pace
    cl |= border & ((x0 + g.xlo < 0) | (x0 + g.xlo > im.width - 2) | (y0 + g.ylo < 0) | (y0 + g.ylo > im.height - 2));
    const int cx = min(max(x0, 0), rowb - 2), cy = min(max(y0, 0), g.ht - 2);
    const int off = cy * rowb + cx;
    const uint32_t vt = tile_pair(tile, off), vb = tile_pair(tile, off + rowb);
    const float i00 = (float)(vt & 255u), i10 = (float)((vt >> 8) & 255u);
    const float i01 = (float)(vb & 255u), i11 = (float)((vb >> 8) & 255u);
    const float top = fmaf(fx, i10 - i00, i00), bot = fmaf(fx, i11 - i01, i01);
    const float val = fmaf(fy, bot - top, top);
    const float a = ((val - o) * tx) * ty;
    s2 = fmaf(a, a, s2);
    s3 = fmaf(a, ty, s3);
    at[i] = a;
    // keep the scheduler from hoisting every row's tile reads (register spills)
    if ((i & 3) == 3) __builtin_amdgcn_sched_barrier(0);
  }
}

// The same samples read straight from memory (clamped reads; uint8 or fp32),
// written to component `dst` of z's rows as they are formed.
template <int N, int IT, int S>
__device__ __forceinline__ void gather_global(float* __restrict__ dst, const RowParam* __restrict__ rp,
                                              const float* __restrict__ taper_s, const swift_image& im, float kux,
                                              float kuy, float o, float tx, int x, int r0, float& s2, float& s3,
                                              bool& cl) {
  s2 = 0.0f;
  s3 = 0.0f;
  const gptr<unsigned char> base = to_global<unsigned char>(im.data);
#pragma unroll 4
  for (int i = 0; i < IT; ++i) {
    const int r = r0 + i;
    const RowParam p = rp[r];
    const float ty = taper_s[r];
    const float xr = p.fx + kux, yr = p.fy + kuy;
    const float xf = floorf(xr), yf = floorf(yr);
    const float fx = xr - xf, fy = yr - yf;
    const int x0 = p.bx + (int)xf, y0 = p.by + (int)yf;
    cl |= (x0 < 0) | (x0 > im.width - 2) | (y0 < 0) | (y0 > im.height - 2);
    const int cx0 = min(max(x0, 0), im.width - 1), cx1 = min(max(x0 + 1, 0), im.width - 1);
    const int cy0 = min(max(y0, 0), im.height - 1), cy1 = min(max(y0 + 1, 0), im.height - 1);
    const gptr<unsigned char> q0 = base + (int64_t)cy0 * im.pitch;
    const gptr<unsigned char> q1 = base + (int64_t)cy1 * im.pitch;
    float i00, i10, i01, i11;
    if (im.dtype == SWIFT_U8) {
      i00 = (float)q0[cx0];
      i10 = (float)q0[cx1];
      i01 = (float)q1[cx0];
      i11 = (float)q1[cx1];
    } else {
      i00 = ((gptr<float>)q0)[cx0];
      i10 = ((gptr<float>)q0)[cx1];
      i01 = ((gptr<float>)q1)[cx0];
      i11 = ((gptr<float>)q1)[cx1];
    }
    const float top = fmaf(fx, i10 - i00, i00), bot = fmaf(fx, i11 - i01, i01);
    const float val = fmaf(fy, bot - top, top);
    const float a = ((val - o) * tx) * ty;
    s2 = fmaf(a, a, s2);
    s3 = fmaf(a, ty, s3);
    dst[2 * (r * S + lidx(x))] = a;
  }
}

template <int N>
__global__ void __launch_bounds__(FusedCfg<N>::NTH) k_fused(MatchArgs a) {
  using C = FftCfg<N>;
  using FC = FusedCfg<N>;
  constexpr int NTH = FC::NTH, S = FC::S, TRW = FC::TRW, TB = FC::TB;
  constexpr int T = C::T, E = C::E, G = NTH / T, NW = NTH / 64, NH = N / 2;
  constexpr int CW = tile_cw<N>();
  constexpr int IT = N * N / NTH;  // gather: consecutive rows per thread
  static_assert(G == NH, "one FFT group per column pair and per row pair");
  static_assert(S >= lidx(N - 1) + 1, "a row holds its FFT scratch");
  static_assert(4 * N * N + 2 * TB + 4 <= N * S * 8 && TB % 16 == 0, "samples of A and both tiles fit in z's storage");
  static_assert(NTH % N == 0 && IT * (NTH / N) == N, "gather layout");
  __shared__ __align__(16) float2 Z[N * S];
  __shared__ RowParam rp[2][N];
  __shared__ float taper_s[N];
  __shared__ float2 tau_s[N];
  __shared__ double red[NW][6];
  __shared__ int redc[NW];
  __shared__ PairStat sps;
  __shared__ float rm1[NW], rm2[NW];
  __shared__ int ri1[NW];
  __shared__ double rs[NW], rq[NW];

  const int tid = threadIdx.x, g = tid / T, t = tid % T, wv = tid >> 6, ln = tid & 63;
  // thread: column x, rows r0 .. r0 + IT - 1 of the gather
  const int x = tid % N, r0 = (tid / N) * IT;
  if (tid < N) {
    taper_s[tid] = a.taper[tid];
    tau_s[tid] = a.tau[tid];
  }
  const int pair = blockIdx.x;
  swift_image im[2];
  RowAffine ra[2];
  TileGeom tg[2];
  bool border[2], trans[2];
  RowParam pt[2];  // translation windows on a tile: the parameters of the thread's first row
  uint4 bufA[TRW], bufB[TRW];
  {
    const int ka = min(max(a.img_a[pair], 0), a.n_imgs - 1);
    const int kb = min(max(a.img_b[pair], 0), a.n_imgs - 1);
    im[0] = a.imgs[ka];
    im[1] = a.imgs[kb];
    ra[0] = row_affine(a.th_a + 8 * (size_t)pair);
    ra[1] = row_affine(a.th_b + 8 * (size_t)pair);
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      im[m].width = max(im[m].width, 2);
      im[m].height = max(im[m].height, 2);
      trans[m] = ra[m].a11 == 1.0 && ra[m].a12 == 0.0 && ra[m].a21 == 0.0 && ra[m].a22 == 1.0;
      if (trans[m]) {
        const double X = fmin(fmax(ra[m].xc, -1e9), 1e9), Y = fmin(fmax(ra[m].yc, -1e9), 1e9);
        const double fxd = floor(X), fyd = floor(Y);
        const bool finite = fabs(X) < 1e8 && fabs(Y) < 1e8;
        const int bx0 = (int)fxd, by0 = (int)fyd;
        tg[m] = tile_geom_trans<N, N, TB, TRW, NW>(bx0, by0, finite, im[m], 0);
        pt[m].bx = bx0 - tg[m].xlo;
        pt[m].by = by0 + (r0 - N / 2) - tg[m].ylo;
        pt[m].fx = (float)(X - fxd);
        pt[m].fy = (float)(Y - fyd);
      } else {
        tg[m] = tile_geom<N, N, TB, TRW, NW>(ra[m], im[m], 0);
        pt[m].bx = pt[m].by = 0;
        pt[m].fx = pt[m].fy = 0.0f;
      }
      border[m] = !(tg[m].use && tg[m].xlo >= 0 && tg[m].xlo + 4 * tg[m].wt4 <= im[m].width && tg[m].ylo >= 0 &&
                    tg[m].ylo + tg[m].ht <= im[m].height);
    }
    // every tile load of both windows in flight before anything waits on them
    if (tg[0].use) tile_fetch<CW, TRW, NW>(bufA, tg[0], im[0], tid);
    if (tg[1].use) tile_fetch<CW, TRW, NW>(bufB, tg[1], im[1], tid);
  }
  // ------------------------------------------------------------ 1. gather
  if (tid < 2 * N && !(tid >= N ? (trans[1] && tg[1].use) : (trans[0] && tg[0].use))) {
    // sampling parameters of row r: integer and fractional parts of the row
    // origin (cx + tx + a12 v, cy + ty + a22 v), v = r - N/2, in FP64; the
    // integer part relative to the tile origin when there is a tile
    const bool mb = tid >= N;
    const int r = tid % N;
    const double xc = mb ? ra[1].xc : ra[0].xc, yc = mb ? ra[1].yc : ra[0].yc;
    const double a12 = mb ? ra[1].a12 : ra[0].a12, a22 = mb ? ra[1].a22 : ra[0].a22;
    const int xo = mb ? (tg[1].use ? tg[1].xlo : 0) : (tg[0].use ? tg[0].xlo : 0);
    const int yo = mb ? (tg[1].use ? tg[1].ylo : 0) : (tg[0].use ? tg[0].ylo : 0);
    const double v = (double)(r - N / 2);
    const double X = fmin(fmax(xc + a12 * v, -1e9), 1e9);
    const double Y = fmin(fmax(yc + a22 * v, -1e9), 1e9);
    const double bxd = floor(X), byd = floor(Y);
    RowParam p;
    p.bx = (int)bxd - xo;
    p.by = (int)byd - yo;
    p.fx = (float)(X - bxd);
    p.fy = (float)(Y - byd);
    rp[mb ? 1 : 0][r] = p;
  }
  const float off[2] = {centre_pixel(im[0], ra[0]), centre_pixel(im[1], ra[1])};
  float* const samp_a = reinterpret_cast<float*>(Z);  // [N][N] samples of A while B is gathered
  uint32_t* const tile0 = reinterpret_cast<uint32_t*>(Z) + N * N;
  uint32_t* const tile1 = tile0 + TB / 4;
  if (tg[0].use) tile_store<CW, TRW, NW>(tile0, bufA, tg[0], im[0], border[0], tid);
  if (tg[1].use) tile_store<CW, TRW, NW>(tile1, bufB, tg[1], im[1], border[1], tid);
  __syncthreads();

  // windows with a tile are gathered while the tiles sit in z's storage (A's
  // samples parked in LDS, B's in registers), then stored into z; windows
  // without one are gathered from memory straight into z afterwards
  float s[6] = {0, 0, 0, 0, 0, 0};
  bool cl = false;
  const float tx = taper_s[x];
  const float u = (float)(x - N / 2);
  float* const zf = reinterpret_cast<float*>(Z);
  if (tg[0].use || tg[1].use) {  // uniform
    float atA[IT], atB[IT];
    float s2, s3;
    if (tg[0].use) {
      gather_tile<N, IT>(atA, tile0, tg[0], trans[0], pt[0], rp[0], taper_s, im[0], border[0], ra[0].f11 * u,
                         ra[0].f21 * u, off[0], tx, x, r0, s2, s3, cl);
      s[1] = s2;
      s[2] = tx * s3;
#pragma unroll
      for (int i = 0; i < IT; ++i) samp_a[(r0 + i) * N + x] = atA[i];
    }
    if (tg[1].use) {
      gather_tile<N, IT>(atB, tile1, tg[1], trans[1], pt[1], rp[1], taper_s, im[1], border[1], ra[1].f11 * u,
                         ra[1].f21 * u, off[1], tx, x, r0, s2, s3, cl);
      s[4] = s2;
      s[5] = tx * s3;
    }
    __syncthreads();  // tiles consumed
    if (tg[0].use) {
#pragma unroll
      for (int i = 0; i < IT; ++i) atA[i] = samp_a[(r0 + i) * N + x];
      __syncthreads();  // parked samples read
    }
    if (tg[0].use && tg[1].use) {
#pragma unroll
      for (int i = 0; i < IT; ++i) Z[(r0 + i) * S + lidx(x)] = make_float2(atA[i], atB[i]);
    } else if (tg[0].use) {
#pragma unroll
      for (int i = 0; i < IT; ++i) zf[2 * ((r0 + i) * S + lidx(x))] = atA[i];
    } else {
#pragma unroll
      for (int i = 0; i < IT; ++i) zf[2 * ((r0 + i) * S + lidx(x)) + 1] = atB[i];
    }
  }
  if (!tg[0].use) {
    float s2, s3;
    gather_global<N, IT, S>(zf, rp[0], taper_s, im[0], ra[0].f11 * u, ra[0].f21 * u, off[0], tx, x, r0, s2, s3, cl);
    s[1] = s2;
    s[2] = tx * s3;
  }
  if (!tg[1].use) {
    float s2, s3;
    gather_global<N, IT, S>(zf + 1, rp[1], taper_s, im[1], ra[1].f11 * u, ra[1].f21 * u, off[1], tx, x, r0, s2, s3,
                            cl);
    s[4] = s2;
    s[5] = tx * s3;
  }
  __syncthreads();

  // ------------------------------------------------------------ 2. row FFTs
  Twiddles<N> tw;
  tw_load<N>(tw, t, a.tw);
  float dcA = 0.0f, dcB = 0.0f;
#pragma unroll 1
  for (int it = 0; it < N / G; ++it) {
    float2* row = Z + (g + it * G) * S;
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
  s[0] = dcA;
  s[3] = dcB;

  // ------------------------------------------------------------ 3. pair statistics
  {
    double acc[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) acc[i] = (double)wave_sum_f32(s[i]);
    const int anyc = __any(cl) ? 1 : 0;
    if (ln == 0) {
#pragma unroll
      for (int i = 0; i < 6; ++i) red[wv][i] = acc[i];
      redc[wv] = anyc;
    }
  }
  __syncthreads();
  // the last wave's lane 0 reduces the statistics while the column transforms
  // start (the whitening below waits for them); wave 0 has the most column work
  if (tid == NTH - 64) {
    double tot[6] = {0, 0, 0, 0, 0, 0};
    int c = 0;
    for (int w = 0; w < NW; ++w) {
#pragma unroll
      for (int i = 0; i < 6; ++i) tot[i] += red[w][i];
      c |= redc[w];
    }
    const PairStat ps = make_pair_stat(tot, c != 0, *a.tinfo, off[0], off[1], N, false, a.p);
    sps = ps;
    if (a.saved_ps) a.saved_ps[pair] = ps;
  }

  // ------------------------------------------------------------ 4. columns
  // Group g > 0 takes column w = g and its mirror N - g; group 0 takes the two
  // self-mirrored columns 0 and N/2 (one more inverse transform, the only
  // divergent step).
  {
    const int w = g, w2 = g == 0 ? NH : N - g;
    float2* cw = Z + lidx(w);
    float2* c2 = Z + lidx(w2);
    float2 v[E], q[E];
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = cw[(t + e * T) * S];
    wave_lds_sync();
    fft_wave_column<N, false>(v, cw, t, tw, S);
#pragma unroll
    for (int e = 0; e < E; ++e) q[e] = c2[(t + e * T) * S];
    wave_lds_sync();
    fft_wave_column<N, false>(q, c2, t, tw, S);
    if (a.saved_Z) {
      float2* sz = a.saved_Z + (size_t)pair * N * N;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        sz[(size_t)w * N + t + e * T] = v[e];
        sz[(size_t)w2 * N + t + e * T] = q[e];
      }
    }
    wave_lds_sync();  // the transforms' scratch reads are done
    // the bins each column's mirror lookups read: column N - g's for column g;
    // for group 0, columns 0 and N/2 are their own mirrors
#pragma unroll
    for (int e = 0; e < E; ++e) c2[(t + e * T) * S] = q[e];
    if (g == 0) {
#pragma unroll
      for (int e = 0; e < E; ++e) cw[(t + e * T) * S] = v[e];
    }
    __syncthreads();  // the pair statistics are in sps
    const PairStat ps = sps;
    const float2* mv = g == 0 ? cw : c2;
    const float2 tauw = tau_s[w], tau2 = tau_s[w2];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int ky = t + e * T, my = ((N - ky) & (N - 1)) * S;
      v[e] = whiten_bin(v[e], cconj(mv[my]), cmul(tau_s[ky], tauw), ps, a.p, a.eps_rel, ky == 0 && w == 0);
      if (g == 0) q[e] = whiten_bin(q[e], cconj(c2[my]), cmul(tau_s[ky], tau2), ps, a.p, a.eps_rel, false);
    }
    wave_lds_sync();  // every lane has read its mirror values
    fft_wave_column<N, true>(v, cw, t, tw, S);
#pragma unroll
    for (int e = 0; e < E; ++e) cw[(t + e * T) * S] = v[e];
    if (g == 0) {
      wave_lds_sync();
      fft_wave_column<N, true>(q, c2, t, tw, S);
#pragma unroll
      for (int e = 0; e < E; ++e) c2[(t + e * T) * S] = q[e];
    }
  }
  __syncthreads();

  // ------------------------------------------------------------ 5. inverse rows
  const int rmax = a.max_shift;  // > 0: the peak is searched within |shift| <= rmax
  Top2 tp;
  tp.m1 = -FLT_MAX;
  tp.i1 = INT_MAX;
  tp.m2 = -FLT_MAX;
  double sum, sq;
  {
    const int ya = 2 * g, yb = ya + 1;
    float2* r1 = Z + ya * S;
    const float2* r2 = r1 + S;
    float2 v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int k = t + e * T;
      float2 g1, g2;
      if (k <= NH) {
        g1 = r1[lidx(k)];
        g2 = r2[lidx(k)];
      } else {
        g1 = cconj(r1[lidx(N - k)]);
        g2 = cconj(r2[lidx(N - k)]);
      }
      v[e] = make_float2(g1.x - g2.y, g1.y + g2.x);
    }
    wave_lds_sync();
    fft_wave<N, true>(v, r1, t, tw);
    // the two surface rows, c(ya, x) and c(yb, x), stay in row ya's storage
#pragma unroll
    for (int e = 0; e < E; ++e) r1[lidx(t + e * T)] = v[e];
    float* surf = a.surfaces ? a.surfaces + (size_t)pair * N * N : nullptr;
    if (surf) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        surf[(size_t)ya * N + t + e * T] = v[e].x;
        surf[(size_t)yb * N + t + e * T] = v[e].y;
      }
    }
    // each lane visits its flat indices in increasing order (row ya, then
    // row yb), so a strict > keeps the first maximum
    const bool ina = rmax == 0 || ya <= rmax || ya >= N - rmax;
    const bool inb = rmax == 0 || yb <= rmax || yb >= N - rmax;
    float ls = 0.0f, lq = 0.0f;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int xx = t + e * T;
      const float ca = v[e].x;
      if (ina && (rmax == 0 || xx <= rmax || xx >= N - rmax)) top2_push_ordered(tp, ca, ya * N + xx);
      ls += ca;
      lq = fmaf(ca, ca, lq);
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int xx = t + e * T;
      const float cb = v[e].y;
      if (inb && (rmax == 0 || xx <= rmax || xx >= N - rmax)) top2_push_ordered(tp, cb, yb * N + xx);
      ls += cb;
      lq = fmaf(cb, cb, lq);
    }
    sum = wave_sum((double)ls);
    sq = wave_sum((double)lq);
  }
  tp = wave_top2(tp);
  if (ln == 0) {
    rm1[wv] = tp.m1;
    ri1[wv] = tp.i1;
    rm2[wv] = tp.m2;
    rs[wv] = sum;
    rq[wv] = sq;
  }
  __syncthreads();

  // ------------------------------------------------------------ 6. record
  if (wv == 0) {
    Top2 b;
    b.m1 = ln < NW ? rm1[ln] : -FLT_MAX;
    b.i1 = ln < NW ? ri1[ln] : INT_MAX;
    b.m2 = ln < NW ? rm2[ln] : -FLT_MAX;
    b = wave_top2(b);
    double tsum = wave_sum(ln < NW ? rs[ln] : 0.0);
    double tsq = wave_sum(ln < NW ? rq[ln] : 0.0);
    const int flat = (b.i1 >= 0 && b.i1 < N * N) ? b.i1 : 0;
    const int iy = flat / N, ix = flat % N;
    // surface value at (y, x): component y & 1 of row (y & ~1)'s storage
    const float* zf = reinterpret_cast<const float*>(Z);
    auto surf_at = [&](int y, int xx) { return zf[2 * ((y & ~1) * S + lidx(xx)) + (y & 1)]; };
    const int R = a.snr_exclude_r;
    double bs = 0.0, bq = 0.0;
    if (R > 0) {
      const int W = 2 * R + 1;
      for (int qd = ln; qd < W * W; qd += 64) {
        const int dy = qd / W - R, dx = qd % W - R;
        const double c = (dx == 0 && dy == 0) ? (double)b.m1 : (double)surf_at((iy + dy) & (N - 1), (ix + dx) & (N - 1));
        bs += c;
        bq += c * c;
      }
      bs = wave_sum(bs);
      bq = wave_sum(bq);
    }
    if (ln == 0) {
      float nb[3][3];
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) nb[dy + 1][dx + 1] = surf_at((iy + dy) & (N - 1), (ix + dx) & (N - 1));
      double count = 0.0;
      // with a search radius the surface sum is taken as exactly 0 (the DC
      // bin of the whitened spectrum is 0), as the five-kernel path does
      if (rmax > 0) tsum = 0.0;
      if (R > 0) {
        // background without the box: N^2 - (2R+1)^2 entries
        tsum -= bs;
        tsq -= bq;
        count = (double)N * (double)N - (double)(2 * R + 1) * (double)(2 * R + 1);
      }
      const PairStat ps = sps;
      swift_match rec = make_record(N, b, tsum, tsq, nb, (ps.flags & 4) ? SWIFT_ST_CLAMPED : 0, count);
      a.out[pair] = rec;
      if (a.saved_rec) a.saved_rec[pair] = rec;
      if (a.saved_nb)
        for (int q = 0; q < 9; ++q) a.saved_nb[(size_t)pair * 9 + q] = nb[q / 3][q % 3];
    }
  }
}

hipError_t launch_fused_group(int n, const MatchArgs& a, hipStream_t s, KernelTimer* kt) {
  if (a.pearson) return hipErrorInvalidValue;
  const unsigned P = (unsigned)a.npairs;
  if (kt) kt->begin("k_fused", n, s);
  switch (n) {
    case 64: k_fused<64><<<P, FusedCfg<64>::NTH, 0, s>>>(a); break;
    case 128: k_fused<128><<<P, FusedCfg<128>::NTH, 0, s>>>(a); break;
    default:
      if (kt) kt->end(s);
      return hipErrorInvalidValue;
  }
  if (kt) kt->end(s);
  return hipGetLastError();
}

}  // namespace swift
