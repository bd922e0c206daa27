// Stack-loop kernels (Sections III-IV): mir rendering of every section by its
// affine, swim window set-up through the affines, and mir's least-squares
// affine of each section from its window matches.
//
// A section affine maps aligned-frame points p to raw-section points q in
// level-0 pixels, q = L p + t, stored as (a11, a12, tx, a21, a22, ty) in FP64.
// A level-l pyramid pixel x_l has its centre at x_0 = 2^l x_l + (2^l - 1)/2.
//
// Rendering decides an integer (round half up of the bilinear value), so the
// coordinate and interpolation arithmetic is FP64 with contraction off: each
// product and sum is rounded on its own, in a fixed order.
#include "swift_dev.hpp"
#include "swift_internal.hpp"

namespace swift {

__device__ __forceinline__ double lvl_to_base(double x, double s, double h) {
#pragma clang fp contract(off)
  return x * s + h;
}
// The level scale s is a power of two, so multiplying by rs = 1/s rounds
// exactly like dividing by s, without an FP64 divide per coordinate.
__device__ __forceinline__ double base_to_lvl(double x, double rs, double h) {
#pragma clang fp contract(off)
  return (x - h) * rs;
}

// Level-l scale 2^l, half-pixel offset (2^l - 1)/2 and reciprocal scale, all
// exact.
struct LevelMap {
  double sc, hf, rs;
  __device__ explicit LevelMap(int level) : sc(ldexp(1.0, level)), hf((sc - 1.0) * 0.5), rs(ldexp(1.0, -level)) {}
};

// Aligned pixel (x, y) of level l through the level-0 affine A = (a11, a12, tx,
// a21, a22, ty): bilinear value of the level-l image at the raw point, clamped
// reads, rounded half up to uint8.
__device__ __forceinline__ uint8_t map_pixel(const uint8_t* __restrict__ img, int64_t spitch, int sw, int sh,
                                             const double* __restrict__ A, const LevelMap& L, int x, int y) {
#pragma clang fp contract(off)
  const double px = lvl_to_base((double)x, L.sc, L.hf), py = lvl_to_base((double)y, L.sc, L.hf);
  const double qx = base_to_lvl(A[0] * px + A[1] * py + A[2], L.rs, L.hf);
  const double qy = base_to_lvl(A[3] * px + A[4] * py + A[5], L.rs, L.hf);
  const double fx0 = floor(qx), fy0 = floor(qy);
  const double fx = qx - fx0, fy = qy - fy0;
  // indices clamped in FP64 first so far-away points cannot overflow an int
  const int x0 = (int)fmin(fmax(fx0, -1.0), (double)sw), y0 = (int)fmin(fmax(fy0, -1.0), (double)sh);
  const int cx0 = min(max(x0, 0), sw - 1), cx1 = min(max(x0 + 1, 0), sw - 1);
  const int cy0 = min(max(y0, 0), sh - 1), cy1 = min(max(y0 + 1, 0), sh - 1);
  const double i00 = img[(int64_t)cy0 * spitch + cx0], i10 = img[(int64_t)cy0 * spitch + cx1];
  const double i01 = img[(int64_t)cy1 * spitch + cx0], i11 = img[(int64_t)cy1 * spitch + cx1];
  const double top = (1.0 - fx) * i00 + fx * i10;
  const double bot = (1.0 - fx) * i01 + fx * i11;
  const double v = (1.0 - fy) * top + fy * bot;
  return (uint8_t)fmin(fmax(floor(v + 0.5), 0.0), 255.0);
}

// ---------------------------------------------------------------- render
// One thread per output pixel; block (x tile, row, section).
__global__ void __launch_bounds__(256) k_render(const uint8_t* __restrict__ src, int64_t spitch, int64_t sstride,
                                                int sw, int sh, const double* __restrict__ aff, int level,
                                                uint8_t* __restrict__ dst, int64_t dpitch, int64_t dstride, int dw) {
  const int x = blockIdx.x * 256 + threadIdx.x;
  const int y = blockIdx.y, s = blockIdx.z;
  if (x >= dw) return;
  const LevelMap L(level);
  dst[(int64_t)s * dstride + (int64_t)y * dpitch + x] =
      map_pixel(src + (int64_t)s * sstride, spitch, sw, sh, aff + 6 * (size_t)s, L, x, y);
}

hipError_t launch_render(const uint8_t* src, int64_t spitch, int64_t sstride, int S, int sh, int sw,
                         const double* aff, int level, uint8_t* dst, int64_t dpitch, int64_t dstride, int dh, int dw,
                         hipStream_t st, KernelTimer* kt) {
  if (S > 0 && dh > 0 && dw > 0) {
    dim3 grid((unsigned)((dw + 255) / 256), (unsigned)dh, (unsigned)S);
    if (kt) kt->begin("k_render", level, st);
    k_render<<<grid, 256, 0, st>>>(src, spitch, sstride, sw, sh, aff, level, dst, dpitch, dstride, dw);
    if (kt) kt->end(st);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- local-affine mesh
// Mesh of one section: nodes at the swim window centres of a grid x grid
// layout of the level-l aligned frame, node (i, j) at (sx/2 + i sx, sy/2 + j
// sy), sx = w_l / grid, sy = h_l / grid.  Cell (ci, cj) is cut along the
// diagonal from node (ci+1, cj) to node (ci, cj+1); triangle 2c holds nodes
// (ci, cj), (ci+1, cj), (ci, cj+1) and triangle 2c+1 the other half, c = cj
// (grid-1) + ci.  A pixel takes the triangle of its cell (clamped to the
// cells, so border triangles extend to the frame edges) on its side of the
// diagonal, the diagonal itself in the first triangle; decided in integers.
struct MeshGeom {
  int g, sx, sy;
  float rsx, rsy;  // 1/sx, 1/sy rounded to float
  MeshGeom(int grid, int h_l, int w_l)
      : g(grid), sx(w_l / grid), sy(h_l / grid), rsx(1.0f / (float)sx), rsy(1.0f / (float)sy) {}
  // floor((v - step/2) / step) clamped to [0, g-2].  |v| < 2^16, so the float
  // quotient is within one of the exact floor; the integer tests correct it.
  __device__ __forceinline__ int cell(int v, int step, float rstep) const {
    const int d = v - step / 2;
    int c = (int)floorf((float)d * rstep);
    c += (c + 1) * step <= d ? 1 : 0;
    c -= c * step > d ? 1 : 0;
    return min(max(c, 0), g - 2);
  }
  __device__ __forceinline__ int triangle(int x, int y) const {
    const int ci = cell(x, sx, rsx), cj = cell(y, sy, rsy);
    const int64_t dx = x - (sx / 2 + ci * sx), dy = y - (sy / 2 + cj * sy);
    const int second = dx * sy + dy * sx > (int64_t)sx * sy ? 1 : 0;
    return 2 * (cj * (g - 1) + ci) + second;
  }
};

// mir texture mapping: each output pixel is rendered by the affine of its
// triangle; tri_aff [S][2 (grid-1)^2][6].  One thread per output pixel.
__global__ void __launch_bounds__(256) k_render_mesh(const uint8_t* __restrict__ src, int64_t spitch,
                                                     int64_t sstride, int sw, int sh,
                                                     const double* __restrict__ tri_aff, MeshGeom M, int level,
                                                     uint8_t* __restrict__ dst, int64_t dpitch, int64_t dstride,
                                                     int dw) {
  const int x = blockIdx.x * 256 + threadIdx.x;
  const int y = blockIdx.y, s = blockIdx.z;
  if (x >= dw) return;
  const int T = 2 * (M.g - 1) * (M.g - 1);
  const double* A = tri_aff + 6 * ((size_t)s * T + M.triangle(x, y));
  const LevelMap L(level);
  dst[(int64_t)s * dstride + (int64_t)y * dpitch + x] =
      map_pixel(src + (int64_t)s * sstride, spitch, sw, sh, A, L, x, y);
}

hipError_t launch_render_mesh(const uint8_t* src, int64_t spitch, int64_t sstride, int S, int sh, int sw,
                              const double* tri_aff, int grid, int level, uint8_t* dst, int64_t dpitch,
                              int64_t dstride, int dh, int dw, hipStream_t st, KernelTimer* kt) {
  if (S > 0 && dh > 0 && dw > 0) {
    dim3 g((unsigned)((dw + 255) / 256), (unsigned)dh, (unsigned)S);
    if (kt) kt->begin("k_render_mesh", level, st);
    k_render_mesh<<<g, 256, 0, st>>>(src, spitch, sstride, sw, sh, tri_aff, MeshGeom(grid, dh, dw), level, dst,
                                     dpitch, dstride, dw);
    if (kt) kt->end(st);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- window set-up
// Window k of section s (row-major grid x grid tiling of the level-l frame):
// B reads the model at the tile centre at identity; A reads the raw section
// around the raw point of that centre with the linear part of A (the
// section's affine, or the affine of the centre's mesh triangle), the centre
// split into a rounded part and a remainder.
__device__ __forceinline__ void window_pair(const double* __restrict__ A, const LevelMap& L, int px, int py,
                                            float* __restrict__ ta, float* __restrict__ tb) {
#pragma clang fp contract(off)
  const double bx = lvl_to_base((double)px, L.sc, L.hf), by = lvl_to_base((double)py, L.sc, L.hf);
  const double cx = base_to_lvl(A[0] * bx + A[1] * by + A[2], L.rs, L.hf);
  const double cy = base_to_lvl(A[3] * bx + A[4] * by + A[5], L.rs, L.hf);
  const double rx = rint(cx), ry = rint(cy);
  ta[0] = (float)rx;
  ta[1] = (float)ry;
  ta[2] = (float)A[0];
  ta[3] = (float)A[1];
  ta[4] = (float)(cx - rx);
  ta[5] = (float)A[3];
  ta[6] = (float)A[4];
  ta[7] = (float)(cy - ry);
  tb[0] = (float)px;
  tb[1] = (float)py;
  tb[2] = 1.0f;
  tb[3] = 0.0f;
  tb[4] = 0.0f;
  tb[5] = 0.0f;
  tb[6] = 1.0f;
  tb[7] = 0.0f;
}

// MESH false: aff [S][6] section affines; MESH true: aff [S][2 (grid-1)^2][6].
template <bool MESH>
__global__ void __launch_bounds__(256) k_stack_windows(int S, const double* __restrict__ aff, int level, int grid,
                                                       int hl, int wl, MeshGeom M, int img_a0, int img_b0,
                                                       float* __restrict__ th_a, float* __restrict__ th_b,
                                                       int32_t* __restrict__ ia, int32_t* __restrict__ ib) {
  const int g2 = grid * grid;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= S * g2) return;
  const int s = i / g2, k = i % g2, gy = k / grid, gx = k % grid;
  const int sx = wl / grid, sy = hl / grid;
  const int px = sx / 2 + gx * sx, py = sy / 2 + gy * sy;
  const double* A;
  if constexpr (MESH) {
    A = aff + 6 * ((size_t)s * (2 * (grid - 1) * (grid - 1)) + M.triangle(px, py));
  } else {
    A = aff + 6 * (size_t)s;
  }
  window_pair(A, LevelMap(level), px, py, th_a + 8 * (size_t)i, th_b + 8 * (size_t)i);
  ia[i] = img_a0 + s;
  ib[i] = img_b0 + s;
}

hipError_t launch_stack_windows(int S, const double* aff, int level, int grid, int hl, int wl, int img_a0,
                                int img_b0, float* th_a, float* th_b, int32_t* ia, int32_t* ib, bool mesh,
                                hipStream_t st) {
  const int n = S * grid * grid;
  if (n > 0) {
    if (mesh)
      k_stack_windows<true><<<(n + 255) / 256, 256, 0, st>>>(S, aff, level, grid, hl, wl, MeshGeom(grid, hl, wl),
                                                             img_a0, img_b0, th_a, th_b, ia, ib);
    else
      k_stack_windows<false><<<(n + 255) / 256, 256, 0, st>>>(S, aff, level, grid, hl, wl, MeshGeom(1, 1, 1),
                                                              img_a0, img_b0, th_a, th_b, ia, ib);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- least-squares affines
// Correspondence of match j: model point p (centre of window B) and raw point
// q (window A's point -d, d the matched shift), both level 0; weight = SNR, or
// 0 for a degenerate window or an SNR below min_snr.
struct Corr {
  double px, py, qx, qy, w;
};
__device__ __forceinline__ Corr correspondence(const float* __restrict__ th_a, const float* __restrict__ th_b,
                                               const swift_match* __restrict__ rec, size_t j, const LevelMap& L,
                                               float min_snr) {
#pragma clang fp contract(off)
  const swift_match r = rec[j];
  const float* a = th_a + 8 * j;
  const float* b = th_b + 8 * j;
  Corr c;
  c.w = ((r.status & SWIFT_ST_DEGENERATE) || !(r.snr >= min_snr)) ? 0.0 : (double)r.snr;
  c.px = lvl_to_base((double)b[0] + (double)b[4], L.sc, L.hf);
  c.py = lvl_to_base((double)b[1] + (double)b[7], L.sc, L.hf);
  c.qx = lvl_to_base((double)a[0] + (double)a[4] - (double)a[2] * r.dx - (double)a[3] * r.dy, L.sc, L.hf);
  c.qy = lvl_to_base((double)a[1] + (double)a[7] - (double)a[5] * r.dx - (double)a[6] * r.dy, L.sc, L.hf);
  return c;
}

// Weighted least-squares affine q ~ L p + t of the correspondences get(i),
// i < count, held by one wave (lane l takes i = l, l + 64, ...), solved on
// centred points: L = (sum w qc pc^T) G^-1 with G = sum w pc pc^T, t = mean q
// - L mean p.  Returns false, and writes nothing, for fewer than three
// weighted points or points on one line; else lane 0 writes out[6].
template <class GET>
__device__ bool wave_fit_affine(int count, GET get, double* __restrict__ out) {
#pragma clang fp contract(off)
  const int ln = threadIdx.x & 63;
  double W = 0.0, Px = 0.0, Py = 0.0, Qx = 0.0, Qy = 0.0, cnt = 0.0;
  for (int i = ln; i < count; i += 64) {
    const Corr c = get(i);
    W += c.w;
    Px += c.w * c.px;
    Py += c.w * c.py;
    Qx += c.w * c.qx;
    Qy += c.w * c.qy;
    cnt += c.w > 0.0 ? 1.0 : 0.0;
  }
  W = wave_sum(W);
  Px = wave_sum(Px);
  Py = wave_sum(Py);
  Qx = wave_sum(Qx);
  Qy = wave_sum(Qy);
  cnt = wave_sum(cnt);
  const double mpx = W > 0.0 ? Px / W : 0.0, mpy = W > 0.0 ? Py / W : 0.0;
  const double mqx = W > 0.0 ? Qx / W : 0.0, mqy = W > 0.0 ? Qy / W : 0.0;
  double gxx = 0.0, gxy = 0.0, gyy = 0.0, sxx = 0.0, sxy = 0.0, syx = 0.0, syy = 0.0;
  for (int i = ln; i < count; i += 64) {
    const Corr c = get(i);
    const double px = c.px - mpx, py = c.py - mpy, qx = c.qx - mqx, qy = c.qy - mqy;
    gxx += c.w * px * px;
    gxy += c.w * px * py;
    gyy += c.w * py * py;
    sxx += c.w * qx * px;
    sxy += c.w * qx * py;
    syx += c.w * qy * px;
    syy += c.w * qy * py;
  }
  gxx = wave_sum(gxx);
  gxy = wave_sum(gxy);
  gyy = wave_sum(gyy);
  sxx = wave_sum(sxx);
  sxy = wave_sum(sxy);
  syx = wave_sum(syx);
  syy = wave_sum(syy);
  const double det = gxx * gyy - gxy * gxy, tr = gxx + gyy;
  if (cnt < 3.0 || !(det > 1e-12 * tr * tr)) return false;
  if (ln == 0) {
    // [a11 a12] = [sxx sxy] G^-1, [a21 a22] = [syx syy] G^-1
    const double a11 = (sxx * gyy - sxy * gxy) / det, a12 = (sxy * gxx - sxx * gxy) / det;
    const double a21 = (syx * gyy - syy * gxy) / det, a22 = (syy * gxx - syx * gxy) / det;
    out[0] = a11;
    out[1] = a12;
    out[2] = mqx - (a11 * mpx + a12 * mpy);
    out[3] = a21;
    out[4] = a22;
    out[5] = mqy - (a21 * mpx + a22 * mpy);
  }
  return true;
}

// mir's affine of each section from its `per` window matches; one wave per
// section.  A singular section keeps its previous affine (status 1).
__global__ void __launch_bounds__(64) k_fit_sections(int per, const float* __restrict__ th_a,
                                                     const float* __restrict__ th_b,
                                                     const swift_match* __restrict__ rec, int level, float min_snr,
                                                     double* __restrict__ aff, int32_t* __restrict__ status) {
  const int s = blockIdx.x;
  const LevelMap L(level);
  const bool ok = wave_fit_affine(
      per, [&](int i) { return correspondence(th_a, th_b, rec, (size_t)s * per + i, L, min_snr); },
      aff + 6 * (size_t)s);
  if (status && threadIdx.x == 0) status[s] = ok ? 0 : 1;
}

hipError_t launch_fit_sections(int S, int per, const float* th_a, const float* th_b, const swift_match* rec,
                               int level, float min_snr, double* aff, int32_t* status, hipStream_t st) {
  if (S > 0) k_fit_sections<<<S, 64, 0, st>>>(per, th_a, th_b, rec, level, min_snr, aff, status);
  return hipGetLastError();
}

// Band of a mesh triangle: its three vertices and every node sharing a mesh
// edge with one of them, as node offsets from the cell's first node (ci, cj);
// twelve for an interior triangle, fewer where the offsets leave the grid.
__constant__ int8_t kBand[2][12][2] = {
    // first triangle: nodes (0,0) (1,0) (0,1)
    {{0, -1}, {1, -1}, {2, -1}, {-1, 0}, {0, 0}, {1, 0}, {2, 0}, {-1, 1}, {0, 1}, {1, 1}, {-1, 2}, {0, 2}},
    // second triangle: nodes (1,0) (1,1) (0,1)
    {{1, -1}, {2, -1}, {0, 0}, {1, 0}, {2, 0}, {-1, 1}, {0, 1}, {1, 1}, {2, 1}, {-1, 2}, {0, 2}, {1, 2}}};

// mir's local affines: one wave per triangle fits the matches of its band
// (pairs s grid^2 + node); a singular triangle takes its section's affine
// (status 1).
__global__ void __launch_bounds__(64) k_fit_mesh(int grid, const float* __restrict__ th_a,
                                                 const float* __restrict__ th_b,
                                                 const swift_match* __restrict__ rec, int level, float min_snr,
                                                 const double* __restrict__ aff, double* __restrict__ tri_aff,
                                                 int32_t* __restrict__ status) {
  const int t = blockIdx.x, s = blockIdx.y;
  const int T = 2 * (grid - 1) * (grid - 1);
  const int c = t >> 1, u = t & 1, ci = c % (grid - 1), cj = c / (grid - 1);
  const LevelMap L(level);
  double* out = tri_aff + 6 * ((size_t)s * T + t);
  const bool ok = wave_fit_affine(
      12,
      [&](int i) {
        const int ni = ci + kBand[u][i][0], nj = cj + kBand[u][i][1];
        if (ni < 0 || nj < 0 || ni >= grid || nj >= grid) return Corr{0.0, 0.0, 0.0, 0.0, 0.0};
        return correspondence(th_a, th_b, rec, (size_t)s * grid * grid + (size_t)nj * grid + ni, L, min_snr);
      },
      out);
  if (threadIdx.x == 0) {
    if (!ok)
      for (int e = 0; e < 6; ++e) out[e] = aff[6 * (size_t)s + e];
    if (status) status[(size_t)s * T + t] = ok ? 0 : 1;
  }
}

hipError_t launch_fit_mesh(int S, int grid, const float* th_a, const float* th_b, const swift_match* rec, int level,
                           float min_snr, const double* aff, double* tri_aff, int32_t* status, hipStream_t st,
                           KernelTimer* kt) {
  const int T = 2 * (grid - 1) * (grid - 1);
  if (S > 0 && T > 0) {
    dim3 g((unsigned)T, (unsigned)S);
    if (kt) kt->begin("k_fit_mesh", grid, st);
    k_fit_mesh<<<g, 64, 0, st>>>(grid, th_a, th_b, rec, level, min_snr, aff, tri_aff, status);
    if (kt) kt->end(st);
  }
  return hipGetLastError();
}

}  // namespace swift
