// Source tiles of the row passes (forward gather and adjoint): the uint8
// footprint of a block's window rows staged in LDS, per-row sampling
// parameters, and the XCD-aware block order.
#pragma once

#include "swift_dev.hpp"

namespace swift {

// Source footprint of one image for the workgroup's R window rows, staged in
// LDS as uint8 rows of wt4 dwords: tile(ty, tx) = img[clamp(ylo + ty)][clamp(xlo + tx)].
// Rows are read in 16-byte chunks: a load instruction of a wave covers
// 64 / CW tile rows of CW chunks each (CW = tile_cw<N>, a power of two).
struct TileGeom {
  int xlo, ylo;   // tile origin in image pixels (xlo a multiple of 16)
  int wt4, ht;    // dwords of footprint per tile row (a multiple of 4), tile rows
  int ts;         // dwords between tile rows in LDS (wt4, or tile_cw * 4 for translation windows)
  bool use;       // the footprint fits the budget and the image allows 16-byte loads
};

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Chunks per tile row: a power of two >= N/16 + 2 (the chunks of a
// translation window's rows), at most 128.  Up to 64 a wave load covers
// 64 / CW whole rows; at 128 (N = 1024) a row takes two wave loads.
template <int N>
__host__ __device__ constexpr int tile_cw() {
  int c = 1;
  while (c < N / 16 + 2 && c < 128) c *= 2;
  return c;
}
// Tile rows per wave load, and wave loads per tile row.
template <int CW> __host__ __device__ constexpr int tile_rpl() { return CW <= 64 ? 64 / CW : 1; }
template <int CW> __host__ __device__ constexpr int tile_lpr() { return CW <= 64 ? 1 : CW / 64; }
// Tile rows that TRW loads per thread of NWV waves cover.
template <int CW, int TRW, int NWV> __host__ __device__ constexpr int tile_rows_cap() {
  return TRW * NWV * tile_rpl<CW>() / tile_lpr<CW>();
}

// Per image and workgroup: affine of the window rows [y0, y0 + R).
struct RowAffine {
  double xc, yc;  // cx + tx, cy + ty
  double a11, a12, a21, a22;
  float f11, f21; // a11, a21 in FP32 for the per-pixel part
};

__device__ __forceinline__ RowAffine row_affine(const float* th) {
  RowAffine r;
  r.xc = (double)th[0] + (double)th[4];
  r.yc = (double)th[1] + (double)th[7];
  r.a11 = th[2];
  r.a12 = th[3];
  r.a21 = th[5];
  r.a22 = th[6];
  r.f11 = th[2];
  r.f21 = th[5];
  return r;
}

// Value of the source pixel nearest the window centre (u = v = 0),
// img[clamp(floor(y + 1/2))][clamp(floor(x + 1/2))]: the offset about which a
// window's samples and sums are formed.
__device__ __forceinline__ float centre_pixel(const swift_image& im, const RowAffine& ra) {
  const double X = fmin(fmax(ra.xc, -1e9), 1e9), Y = fmin(fmax(ra.yc, -1e9), 1e9);
  const int x = (int)fmin(fmax(floor(X + 0.5), 0.0), (double)(im.width - 1));
  const int y = (int)fmin(fmax(floor(Y + 0.5), 0.0), (double)(im.height - 1));
  const gptr<unsigned char> row = to_global<unsigned char>(im.data) + (int64_t)y * im.pitch;
  return im.dtype == SWIFT_U8 ? (float)row[x] : ((gptr<float>)row)[x];
}

// NWV: waves of the workgroup that fetch the tile (tile_fetch).
template <int N, int R, int BUDGET, int TRW, int NWV = 4>
__device__ __forceinline__ TileGeom tile_geom(const RowAffine& ra, const swift_image& im, int y0) {
  TileGeom g;
  const double ulo = -N / 2, uhi = N / 2 - 1;
  const double vlo = y0 - N / 2, vhi = y0 + R - 1 - N / 2;
  const double xmin = ra.xc + fmin(ra.a11 * ulo, ra.a11 * uhi) + fmin(ra.a12 * vlo, ra.a12 * vhi);
  const double xmax = ra.xc + fmax(ra.a11 * ulo, ra.a11 * uhi) + fmax(ra.a12 * vlo, ra.a12 * vhi);
  const double ymin = ra.yc + fmin(ra.a21 * ulo, ra.a21 * uhi) + fmin(ra.a22 * vlo, ra.a22 * vhi);
  const double ymax = ra.yc + fmax(ra.a21 * ulo, ra.a21 * uhi) + fmax(ra.a22 * vlo, ra.a22 * vhi);
  const bool finite = fabs(xmin) < 1e8 && fabs(xmax) < 1e8 && fabs(ymin) < 1e8 && fabs(ymax) < 1e8;
  g.use = false;
  g.xlo = g.ylo = 0;
  g.wt4 = g.ht = g.ts = 0;
  // every 16-byte chunk is either inside the image or wholly outside it
  if (BUDGET == 0 || !finite || im.dtype != SWIFT_U8 || im.width < 16 || (im.width & 15) || (im.pitch & 15) ||
      (((uintptr_t)im.data) & 15))
    return g;
  // one pixel of margin on both sides absorbs FP32 rounding of the per-pixel coordinates
  const int xl = (int)floor(xmin) - 1, xh = (int)floor(xmax) + 2;
  const int yl = (int)floor(ymin) - 1, yh = (int)floor(ymax) + 2;
  g.xlo = xl - (((xl % 16) + 16) % 16);
  g.ylo = yl;
  const int w16 = (xh - g.xlo + 16) / 16;
  g.wt4 = 4 * w16;
  g.ts = g.wt4;
  g.ht = yh - yl + 1;
  constexpr int CW = tile_cw<N>();
  g.use = (long long)w16 * 16 * g.ht <= BUDGET && g.ht <= tile_rows_cap<CW, TRW, NWV>() && w16 <= CW;
  return g;
}

// tile_geom for a translation window (identity linear part): the footprint of
// rows [y0, y0 + R) is x in [xc - N/2, xc + N/2 - 1], y in [yc + y0 - N/2,
// yc + y0 + R - 1 - N/2], so with bx0 = floor(xc), by0 = floor(yc) the
// geometry is integer arithmetic (the same footprint as tile_geom's).  Its
// LDS rows are a fixed tile_cw<N> chunks apart, so the gather addresses
// every row at a constant offset.
template <int N, int R, int BUDGET, int TRW, int NWV = 4>
__device__ __forceinline__ TileGeom tile_geom_trans(int bx0, int by0, bool finite, const swift_image& im, int y0) {
  TileGeom g;
  g.use = false;
  g.xlo = g.ylo = 0;
  g.wt4 = g.ht = g.ts = 0;
  if (BUDGET == 0 || !finite || im.dtype != SWIFT_U8 || im.width < 16 || (im.width & 15) || (im.pitch & 15) ||
      (((uintptr_t)im.data) & 15))
    return g;
  const int xl = bx0 - N / 2 - 1, xh = bx0 + N / 2 + 1;
  const int yl = by0 + y0 - N / 2 - 1, yh = by0 + y0 + R + 1 - N / 2;
  g.xlo = xl - (((xl % 16) + 16) % 16);
  g.ylo = yl;
  const int w16 = (xh - g.xlo + 16) / 16;
  g.wt4 = 4 * w16;
  g.ht = yh - yl + 1;
  constexpr int CW = tile_cw<N>();
  g.ts = 4 * CW;
  g.use = CW * 16 * g.ht <= BUDGET && g.ht <= tile_rows_cap<CW, TRW, NWV>() && w16 <= CW;
  return g;
}

// Tiles are fetched in two steps so all loads are in flight at once:
// tile_fetch issues every global load of a thread into registers and nothing
// consumes them until tile_store writes them to LDS.  With CW <= 64, lane l
// of wave w takes chunk c = l % CW of tile row (NWV j + w) (64 / CW) + l / CW
// in load j; with CW = 128, loads 2i and 2i + 1 take chunks l and l + 64 of
// tile row NWV i + w (rows past the tile repeat its last row, which the cache
// serves).  Loads are unconditional and in bounds: rows are clamped into the
// image and a chunk left or right of the image is read at the nearest
// in-image chunk; on workgroups whose tile crosses the border, tile_store
// replaces such a chunk by its edge byte repeated, so byte i holds
// img[clamp(y)][clamp(x + i)].
template <int CW>
__device__ __forceinline__ void tile_slot(int j, int wv, int ln, int nwv, int& ty, int& c) {
  constexpr int RPL = tile_rpl<CW>(), LPR = tile_lpr<CW>();
  if constexpr (LPR == 1) {
    c = ln % CW;
    ty = (nwv * j + wv) * RPL + ln / CW;
  } else {
    c = ln + 64 * (j % LPR);
    ty = nwv * (j / LPR) + wv;
  }
}

template <int CW, int RW, int NWV = 4>
__device__ __forceinline__ void tile_fetch(uint4 (&buf)[RW], const TileGeom& g, const swift_image& im, int tid) {
  const gptr<unsigned char> base = to_global<unsigned char>(im.data);
  // the wave index is uniform: with one tile row per load the row address is
  // scalar and a load adds only the lane's 32-bit offset
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6), ln = tid & 63;
#pragma unroll
  for (int j = 0; j < RW; ++j) {
    int ty, c;
    tile_slot<CW>(j, wv, ln, NWV, ty, c);
    const uint32_t xc = (uint32_t)min(max(g.xlo + 16 * c, 0), im.width - 16);
    const int yy = min(max(g.ylo + min(ty, g.ht - 1), 0), im.height - 1);
    const gptr<unsigned char> row = base + (int64_t)yy * im.pitch;
    const u32x4 v = *(gptr<u32x4>)(row + xc);
    buf[j] = make_uint4(v.x, v.y, v.z, v.w);
  }
}

template <int CW, int RW, int NWV = 4>
__device__ __forceinline__ void tile_store(uint32_t* __restrict__ tile, const uint4 (&buf)[RW], const TileGeom& g,
                                           const swift_image& im, bool border, int tid) {
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6), ln = tid & 63;
#pragma unroll
  for (int j = 0; j < RW; ++j) {
    int ty, c;
    tile_slot<CW>(j, wv, ln, NWV, ty, c);
    const int x = g.xlo + 16 * c;
    const bool left = border && x < 0, right = border && x >= im.width;
    if (ty < g.ht && 4 * c < g.ts) {
      uint4 v = buf[j];
      if (left | right) {
        const uint32_t sp = (left ? (v.x & 255u) : (v.w >> 24)) * 0x01010101u;
        v = make_uint4(sp, sp, sp, sp);
      }
      *reinterpret_cast<uint4*>(tile + ty * g.ts + 4 * c) = v;
    }
  }
}

// Row stride (float2) of the forward stage: at least a transform's scratch,
// and chosen so that the read-out in 8-row tiles hits distinct bank pairs: a
// thread takes rows r and r + 1 of one bin, and the 32 lanes of an 8-byte
// access span RP row pairs and 32 / RP consecutive bins, so the offsets
// 2 p RS (p < RP) must be distinct multiples of 32 / RP modulo 32, i.e.
// RS = 16 / RP (mod 32 / RP).
template <int N, int R>
__host__ __device__ constexpr int fwd_stride() {
  const int RP = R >= 8 ? 4 : R / 2;
  int rs = fft_scratch<N>();
  while (rs % (32 / RP) != 16 / RP) ++rs;
  return rs;
}

// Row stride (float2) of a stage that thread r = tid % R fills at consecutive
// columns (the 32 lanes of an 8-byte access span R' = min(R, 32) rows and
// 32 / R' columns): at least `need`, and an odd multiple of 32 / R', so that
// those lanes hit distinct bank pairs.
template <int R>
__host__ __device__ constexpr int rows_stride(int need) {
  const int Rp = R < 32 ? R : 32;
  int rs = need;
  while (rs % (64 / Rp) != 32 / Rp) ++rs;
  return rs;
}

// Per-row sampling parameters of one image, computed once per workgroup: the
// row's coordinate at u = 0 split into an integer part (relative to the tile
// origin when a tile is used) and an FP32 fraction, so the per-pixel work is
// FP32 on small numbers while the absolute position keeps FP64 precision.
struct RowParam {
  int bx, by;      // integer part (tile-relative on the tile path)
  float fx, fy;    // fractional part in [0, 1)
};

// Bytes off and off + 1 of the LDS tile in the low half of a word.  Lanes
// reading neighbouring bytes share dwords; byte-wide LDS reads of one dword by
// several lanes serialise, dword reads of one dword do not, so the pair is
// cut out of the two aligned dwords that hold it.
__device__ __forceinline__ uint32_t tile_pair(const uint32_t* __restrict__ tile, int off) {
  const uint32_t* w = tile + (off >> 2);
  return __builtin_amdgcn_alignbyte(w[1], w[0], (uint32_t)(off & 3));
}

template <int N> struct GatherCfg {
  static constexpr int XV = N >= 256 ? N / 256 : 1;   // columns per thread and row
  static constexpr int RPI = N >= 256 ? 1 : 256 / N;  // rows per iteration
};


// Block order for launches of many independent blocks: consecutive blocks of
// one pair go to the same XCD (the hardware deals blocks round-robin over
// the 8 XCDs), so a pair's source rows and tiles share one L2.
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int per = nb >> 3, full = per << 3;
  return b >= full ? b : (b & 7) * per + (b >> 3);
}

}  // namespace swift
