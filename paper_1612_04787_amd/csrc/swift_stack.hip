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
__device__ __forceinline__ double base_to_lvl(double x, double s, double h) {
#pragma clang fp contract(off)
  return (x - h) / s;
}

// ---------------------------------------------------------------- render
// One thread per output pixel; block (x tile, row, section).
__global__ void __launch_bounds__(256) k_render(const uint8_t* __restrict__ src, int64_t spitch, int64_t sstride,
                                                int sw, int sh, const double* __restrict__ aff, int level,
                                                uint8_t* __restrict__ dst, int64_t dpitch, int64_t dstride, int dw) {
#pragma clang fp contract(off)
  const int x = blockIdx.x * 256 + threadIdx.x;
  const int y = blockIdx.y, s = blockIdx.z;
  if (x >= dw) return;
  const double* A = aff + 6 * (size_t)s;
  const double sc = (double)(1 << level), hf = (sc - 1.0) / 2.0;
  const double px = lvl_to_base((double)x, sc, hf), py = lvl_to_base((double)y, sc, hf);
  const double qx = base_to_lvl(A[0] * px + A[1] * py + A[2], sc, hf);
  const double qy = base_to_lvl(A[3] * px + A[4] * py + A[5], sc, hf);
  const double fx0 = floor(qx), fy0 = floor(qy);
  const double fx = qx - fx0, fy = qy - fy0;
  // indices clamped in FP64 first so far-away points cannot overflow an int
  const int x0 = (int)fmin(fmax(fx0, -1.0), (double)sw), y0 = (int)fmin(fmax(fy0, -1.0), (double)sh);
  const int cx0 = min(max(x0, 0), sw - 1), cx1 = min(max(x0 + 1, 0), sw - 1);
  const int cy0 = min(max(y0, 0), sh - 1), cy1 = min(max(y0 + 1, 0), sh - 1);
  const uint8_t* img = src + (int64_t)s * sstride;
  const double i00 = img[(int64_t)cy0 * spitch + cx0], i10 = img[(int64_t)cy0 * spitch + cx1];
  const double i01 = img[(int64_t)cy1 * spitch + cx0], i11 = img[(int64_t)cy1 * spitch + cx1];
  const double top = (1.0 - fx) * i00 + fx * i10;
  const double bot = (1.0 - fx) * i01 + fx * i11;
  const double v = (1.0 - fy) * top + fy * bot;
  const double r = fmin(fmax(floor(v + 0.5), 0.0), 255.0);
  dst[(int64_t)s * dstride + (int64_t)y * dpitch + x] = (uint8_t)r;
}

hipError_t launch_render(const uint8_t* src, int64_t spitch, int64_t sstride, int S, int sh, int sw,
                         const double* aff, int level, uint8_t* dst, int64_t dpitch, int64_t dstride, int dh, int dw,
                         hipStream_t st) {
  if (S > 0 && dh > 0 && dw > 0) {
    dim3 grid((unsigned)((dw + 255) / 256), (unsigned)dh, (unsigned)S);
    k_render<<<grid, 256, 0, st>>>(src, spitch, sstride, sw, sh, aff, level, dst, dpitch, dstride, dw);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------- window set-up
// Window k of section s (row-major grid x grid tiling of the level-l frame):
// B reads the model at the tile centre at identity; A reads the raw section
// around the raw point of that centre with the section's linear part, the
// centre split into a rounded part and a remainder.
__global__ void __launch_bounds__(256) k_stack_windows(int S, const double* __restrict__ aff, int level, int grid,
                                                       int hl, int wl, int img_a0, int img_b0,
                                                       float* __restrict__ th_a, float* __restrict__ th_b,
                                                       int32_t* __restrict__ ia, int32_t* __restrict__ ib) {
#pragma clang fp contract(off)
  const int g2 = grid * grid;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= S * g2) return;
  const int s = i / g2, k = i % g2, gy = k / grid, gx = k % grid;
  const int sx = wl / grid, sy = hl / grid;
  const int px = sx / 2 + gx * sx, py = sy / 2 + gy * sy;
  const double* A = aff + 6 * (size_t)s;
  const double sc = (double)(1 << level), hf = (sc - 1.0) / 2.0;
  const double bx = lvl_to_base((double)px, sc, hf), by = lvl_to_base((double)py, sc, hf);
  const double cx = base_to_lvl(A[0] * bx + A[1] * by + A[2], sc, hf);
  const double cy = base_to_lvl(A[3] * bx + A[4] * by + A[5], sc, hf);
  const double rx = rint(cx), ry = rint(cy);
  float* ta = th_a + 8 * (size_t)i;
  float* tb = th_b + 8 * (size_t)i;
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
  ia[i] = img_a0 + s;
  ib[i] = img_b0 + s;
}

hipError_t launch_stack_windows(int S, const double* aff, int level, int grid, int hl, int wl, int img_a0,
                                int img_b0, float* th_a, float* th_b, int32_t* ia, int32_t* ib, hipStream_t st) {
  const int n = S * grid * grid;
  if (n > 0)
    k_stack_windows<<<(n + 255) / 256, 256, 0, st>>>(S, aff, level, grid, hl, wl, img_a0, img_b0, th_a, th_b, ia,
                                                     ib);
  return hipGetLastError();
}

// ---------------------------------------------------------------- per-section affine fit
// One wave per section.  Correspondence i: model point p (centre of window B)
// and raw point q (window A's point -d, d the matched shift), both level 0;
// weight = SNR, or 0 for a degenerate window or an SNR below min_snr.  The
// weighted least-squares affine q ~ L p + t is solved on centred points:
// L = (sum w qc pc^T) G^-1 with G = sum w pc pc^T, t = mean q - L mean p.
__global__ void __launch_bounds__(64) k_fit_sections(int per, const float* __restrict__ th_a,
                                                     const float* __restrict__ th_b,
                                                     const swift_match* __restrict__ rec, int level, float min_snr,
                                                     double* __restrict__ aff, int32_t* __restrict__ status) {
#pragma clang fp contract(off)
  const int s = blockIdx.x, ln = threadIdx.x;
  const double sc = (double)(1 << level), hf = (sc - 1.0) / 2.0;
  double W = 0.0, Px = 0.0, Py = 0.0, Qx = 0.0, Qy = 0.0, cnt = 0.0;
  for (int i = ln; i < per; i += 64) {
    const size_t j = (size_t)s * per + i;
    const swift_match r = rec[j];
    const double w = ((r.status & SWIFT_ST_DEGENERATE) || !(r.snr >= min_snr)) ? 0.0 : (double)r.snr;
    const float* a = th_a + 8 * j;
    const float* b = th_b + 8 * j;
    const double px = lvl_to_base((double)b[0] + (double)b[4], sc, hf);
    const double py = lvl_to_base((double)b[1] + (double)b[7], sc, hf);
    const double qx = lvl_to_base((double)a[0] + (double)a[4] - (double)a[2] * r.dx - (double)a[3] * r.dy, sc, hf);
    const double qy = lvl_to_base((double)a[1] + (double)a[7] - (double)a[5] * r.dx - (double)a[6] * r.dy, sc, hf);
    W += w;
    Px += w * px;
    Py += w * py;
    Qx += w * qx;
    Qy += w * qy;
    cnt += w > 0.0 ? 1.0 : 0.0;
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
  for (int i = ln; i < per; i += 64) {
    const size_t j = (size_t)s * per + i;
    const swift_match r = rec[j];
    const double w = ((r.status & SWIFT_ST_DEGENERATE) || !(r.snr >= min_snr)) ? 0.0 : (double)r.snr;
    const float* a = th_a + 8 * j;
    const float* b = th_b + 8 * j;
    const double px = lvl_to_base((double)b[0] + (double)b[4], sc, hf) - mpx;
    const double py = lvl_to_base((double)b[1] + (double)b[7], sc, hf) - mpy;
    const double qx =
        lvl_to_base((double)a[0] + (double)a[4] - (double)a[2] * r.dx - (double)a[3] * r.dy, sc, hf) - mqx;
    const double qy =
        lvl_to_base((double)a[1] + (double)a[7] - (double)a[5] * r.dx - (double)a[6] * r.dy, sc, hf) - mqy;
    gxx += w * px * px;
    gxy += w * px * py;
    gyy += w * py * py;
    sxx += w * qx * px;
    sxy += w * qx * py;
    syx += w * qy * px;
    syy += w * qy * py;
  }
  gxx = wave_sum(gxx);
  gxy = wave_sum(gxy);
  gyy = wave_sum(gyy);
  sxx = wave_sum(sxx);
  sxy = wave_sum(sxy);
  syx = wave_sum(syx);
  syy = wave_sum(syy);
  if (ln == 0) {
    double* A = aff + 6 * (size_t)s;
    const double det = gxx * gyy - gxy * gxy, tr = gxx + gyy;
    if (cnt < 3.0 || !(det > 1e-12 * tr * tr)) {
      if (status) status[s] = 1;  // keep the previous affine
      return;
    }
    // [a11 a12] = [sxx sxy] G^-1, [a21 a22] = [syx syy] G^-1
    const double a11 = (sxx * gyy - sxy * gxy) / det, a12 = (sxy * gxx - sxx * gxy) / det;
    const double a21 = (syx * gyy - syy * gxy) / det, a22 = (syy * gxx - syx * gxy) / det;
    A[0] = a11;
    A[1] = a12;
    A[2] = mqx - (a11 * mpx + a12 * mpy);
    A[3] = a21;
    A[4] = a22;
    A[5] = mqy - (a21 * mpx + a22 * mpy);
    if (status) status[s] = 0;
  }
}

hipError_t launch_fit_sections(int S, int per, const float* th_a, const float* th_b, const swift_match* rec,
                               int level, float min_snr, double* aff, int32_t* status, hipStream_t st) {
  if (S > 0) k_fit_sections<<<S, 64, 0, st>>>(per, th_a, th_b, rec, level, min_snr, aff, status);
  return hipGetLastError();
}

}  // namespace swift
