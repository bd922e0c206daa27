// Source tiles of the row passes (forward gather and adjoint): the uint8
// footprint of a block's window rows staged in LDS, per-row sampling
// parameters, and the XCD-aware block order.
#pragma once

#include "swift_dev.hpp"

namespace swift {

// Source footprint of one image for the workgroup's R window rows, staged in
// LDS as uint8 rows of wt4 dwords: tile(ty, tx) = img[clamp(ylo + ty)][clamp(xlo + tx)].
struct TileGeom {
  int xlo, ylo;   // tile origin in image pixels (xlo a multiple of 4)
  int wt4, ht;    // dwords per tile row, tile rows
  bool use;       // the footprint fits the budget and the image allows dword loads
};

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

__device__ __forceinline__ int floor_to4(int v) { return v - (((v % 4) + 4) % 4); }

template <int N, int R, int BUDGET, int TRW, int TMC>
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
  g.wt4 = g.ht = 0;
  if (BUDGET == 0 || !finite || im.dtype != SWIFT_U8 || (im.pitch & 3) || (im.width & 3) ||
      (((uintptr_t)im.data) & 3))
    return g;
  // one pixel of margin on both sides absorbs FP32 rounding of the per-pixel coordinates
  const int xl = (int)floor(xmin) - 1, xh = (int)floor(xmax) + 2;
  const int yl = (int)floor(ymin) - 1, yh = (int)floor(ymax) + 2;
  g.xlo = floor_to4(xl);
  g.ylo = yl;
  g.wt4 = (xh - g.xlo + 4) / 4;
  g.ht = yh - yl + 1;
  g.use = (long long)g.wt4 * 4 * g.ht <= BUDGET && g.ht <= 4 * TRW && g.wt4 <= 64 * TMC;
  return g;
}

// Tile dwords are fetched in two steps so all loads are in flight at once:
// tile_fetch issues every global load of a thread into registers and nothing
// consumes them until tile_store writes them to LDS.  Wave w fetches tile rows
// w + 4 j, lane l dword columns l + 64 c.  Loads are unconditional (coordinates
// clamped into the image, so every load is in bounds; a branch between a load
// and its use would make the compiler drain the load queue); only in-range
// elements are stored.  Border dwords are read at the nearest in-image
// aligned dword and, on workgroups whose tile crosses the image border, their
// bytes re-selected with v_perm so that byte i holds img[y][clamp(x + i)].
template <int RW, int MC>
__device__ __forceinline__ void tile_fetch(uint32_t (&buf)[RW][MC], const TileGeom& g, const swift_image& im,
                                           int tid) {
  const gptr<unsigned char> base = to_global<unsigned char>(im.data);
  const int wv = tid >> 6, ln = tid & 63;
  int xc[MC];
#pragma unroll
  for (int c = 0; c < MC; ++c) xc[c] = min(max(g.xlo + 4 * (ln + 64 * c), 0), im.width - 4);
#pragma unroll
  for (int j = 0; j < RW; ++j) {
    const int yy = min(max(g.ylo + wv + 4 * j, 0), im.height - 1);
    const gptr<unsigned char> row = base + (int64_t)yy * im.pitch;
#pragma unroll
    for (int c = 0; c < MC; ++c) buf[j][c] = *(gptr<uint32_t>)(row + xc[c]);
  }
}

template <int RW, int MC>
__device__ __forceinline__ void tile_store(uint32_t* __restrict__ tile, const uint32_t (&buf)[RW][MC],
                                           const TileGeom& g, const swift_image& im, bool border, int tid) {
  const int wv = tid >> 6, ln = tid & 63;
  uint32_t sel[MC];
#pragma unroll
  for (int c = 0; c < MC; ++c) {
    const int xx = g.xlo + 4 * (ln + 64 * c);
    const int xc = min(max(xx, 0), im.width - 4);
    sel[c] = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) sel[c] |= (uint32_t)(min(max(xx + b, 0), im.width - 1) - xc) << (8 * b);
  }
#pragma unroll
  for (int j = 0; j < RW; ++j) {
    const int ty = wv + 4 * j;
#pragma unroll
    for (int c = 0; c < MC; ++c) {
      const int tx4 = ln + 64 * c;
      if (ty < g.ht && tx4 < g.wt4)
        tile[ty * g.wt4 + tx4] = border ? __builtin_amdgcn_perm(buf[j][c], buf[j][c], sel[c]) : buf[j][c];
    }
  }
}

// Row stride (float2) of the forward stage: >= lidx(N), chosen so that the
// transposed read-out (rows fastest) hits distinct LDS banks.
template <int N, int R>
__host__ __device__ constexpr int fwd_stride() {
  const int target = R >= 16 ? 1 : 16 / R;
  int rs = lidx(N);
  while ((rs & 15) != target) ++rs;
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
