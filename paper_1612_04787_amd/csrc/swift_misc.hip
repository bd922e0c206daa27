// Scoring of given surfaces, z-projection models and the x2 pyramid.
#include "swift_dev.hpp"

namespace swift {

// ---------------------------------------------------------------- scoring (Z-score of the peak)
// One workgroup per surface: first maximum, top-2 margin, FP64 sum and sum of
// squares, then the record with the 3x3 centroid read from the surface.
__global__ void __launch_bounds__(256) k_snr(const float* __restrict__ surf, int n, int R, swift_match* out) {
  __shared__ float rm1[4], rm2[4];
  __shared__ int ri1[4];
  __shared__ double rs[4], rq[4];
  __shared__ float nb[3][3];
  const float* s = surf + (size_t)blockIdx.x * n * n;
  const int tid = threadIdx.x;
  Top2 tp;
  tp.m1 = -FLT_MAX;
  tp.i1 = INT_MAX;
  tp.m2 = -FLT_MAX;
  double sum = 0.0, sq = 0.0;
  for (int i = tid; i < n * n; i += 256) {
    const float v = s[i];
    top2_push(tp, v, i);
    sum += (double)v;
    sq += (double)v * (double)v;
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
    const int flat = (b.i1 >= 0 && b.i1 < n * n) ? b.i1 : 0;
    const int iy = flat / n, ix = flat % n;
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx)
        nb[dy + 1][dx + 1] = s[(size_t)((iy + dy + n) % n) * n + ((ix + dx + n) % n)];
    double sum = rs[0] + rs[1] + rs[2] + rs[3], sq = rq[0] + rq[1] + rq[2] + rq[3], count = 0.0;
    if (R > 0) {
      // the background leaves out the (2R+1)^2 box around the peak
      for (int dy = -R; dy <= R; ++dy)
        for (int dx = -R; dx <= R; ++dx) {
          const double c = (double)s[(size_t)(((iy + dy) % n + n) % n) * n + (((ix + dx) % n + n) % n)];
          sum -= c;
          sq -= c * c;
        }
      count = (double)n * (double)n - (double)(2 * R + 1) * (double)(2 * R + 1);
    }
    out[blockIdx.x] = make_record(n, b, sum, sq, nb, 0, count);
  }
}

hipError_t launch_snr(const float* surf, int n, int batch, int exclude_r, swift_match* out, hipStream_t st) {
  if (batch > 0) k_snr<<<batch, 256, 0, st>>>(surf, n, exclude_r, out);
  return hipGetLastError();
}

template <int SIDE>
hipError_t launch_project_sel(const uint8_t* src, int64_t pitch, int64_t sstride, int S, int H, int W,
                              const uint8_t* excl, int k, uint8_t* dst, int64_t dpitch, int64_t dstride,
                              hipStream_t st);

// ---------------------------------------------------------------- z-projection model
// Each thread owns BW consecutive pixels of one row and walks the stack in z,
// keeping the 2K+1 sections around s in registers, so every section byte is
// read once.  out[s] = (2 S + n) / (2 n) rounded down = the round-half-up mean
// of the n included neighbours (exact: the quotient is formed in FP32 with a
// 1/(4n) guard that no rounding error can cross for n <= 16).
template <int BW> struct Pix;
template <> struct Pix<16> { using T = uint4; };
template <> struct Pix<1> { using T = unsigned char; };

__device__ __forceinline__ uint32_t div_pack4(uint32_t lo, uint32_t hi, float inv2n, uint32_t nn) {
  // lo holds 16-bit sums of bytes 0 and 2, hi of bytes 1 and 3
  const uint32_t s0 = lo & 0xFFFFu, s2 = lo >> 16, s1 = hi & 0xFFFFu, s3 = hi >> 16;
  const uint32_t q0 = (uint32_t)floorf(((float)(2u * s0 + nn) + 0.5f) * inv2n);
  const uint32_t q1 = (uint32_t)floorf(((float)(2u * s1 + nn) + 0.5f) * inv2n);
  const uint32_t q2 = (uint32_t)floorf(((float)(2u * s2 + nn) + 0.5f) * inv2n);
  const uint32_t q3 = (uint32_t)floorf(((float)(2u * s3 + nn) + 0.5f) * inv2n);
  return q0 | (q1 << 8) | (q2 << 16) | (q3 << 24);
}

// SIDE 0: the two-sided model (neighbours on both sides); SIDE -1 / +1: the
// one-sided models of jump repair (only the k sections before / after).
template <int K, int BW, int SIDE>
__global__ void __launch_bounds__(256) k_project(const uint8_t* __restrict__ src, int64_t pitch, int64_t sstride,
                                                 int S, int H, int W, const uint8_t* __restrict__ excl,
                                                 uint8_t* __restrict__ dst, int64_t dpitch, int64_t dstride) {
  using PT = typename Pix<BW>::T;
  constexpr int WN = 2 * K + 1;
  const int cpr = W / BW;
  const long long gid = (long long)blockIdx.x * 256 + threadIdx.x;
  if (gid >= (long long)H * cpr) return;
  const int y = (int)(gid / cpr), x = (int)(gid % cpr) * BW;
  const uint8_t* col = src + (int64_t)y * pitch + x;
  uint8_t* ocol = dst + (int64_t)y * dpitch + x;

  PT win[WN];
#pragma unroll
  for (int i = 0; i < WN; ++i) {
    const int j = i - K;
    if (j >= 0 && j < S) win[i] = *(const PT*)(col + (int64_t)j * sstride);
    else win[i] = PT{};
  }
  for (int s = 0; s < S; ++s) {
    uint32_t nn = 0;
    if constexpr (BW == 16) {
      uint32_t lo[4] = {0, 0, 0, 0}, hi[4] = {0, 0, 0, 0};
#pragma unroll
      for (int i = 0; i < WN; ++i) {
        const int j = s - K + i;
        if (i != K && (SIDE == 0 || (SIDE < 0 ? i < K : i > K)) && j >= 0 && j < S && !(excl && excl[j])) {
          ++nn;
          const uint4 v = win[i];
          const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            lo[q] += w4[q] & 0x00FF00FFu;
            hi[q] += (w4[q] >> 8) & 0x00FF00FFu;
          }
        }
      }
      uint4 o = make_uint4(0, 0, 0, 0);
      if (nn > 0) {
        const float inv2n = 1.0f / (float)(2u * nn);
        o.x = div_pack4(lo[0], hi[0], inv2n, nn);
        o.y = div_pack4(lo[1], hi[1], inv2n, nn);
        o.z = div_pack4(lo[2], hi[2], inv2n, nn);
        o.w = div_pack4(lo[3], hi[3], inv2n, nn);
      }
      *(uint4*)(ocol + (int64_t)s * dstride) = o;
    } else {
      uint32_t acc = 0;
#pragma unroll
      for (int i = 0; i < WN; ++i) {
        const int j = s - K + i;
        if (i != K && (SIDE == 0 || (SIDE < 0 ? i < K : i > K)) && j >= 0 && j < S && !(excl && excl[j])) {
          ++nn;
          acc += win[i];
        }
      }
      uint8_t o = 0;
      if (nn > 0) o = (uint8_t)floorf(((float)(2u * acc + nn) + 0.5f) / (float)(2u * nn));
      ocol[(int64_t)s * dstride] = o;
    }
#pragma unroll
    for (int i = 0; i < WN - 1; ++i) win[i] = win[i + 1];
    const int jn = s + K + 1;
    if (jn < S) win[WN - 1] = *(const PT*)(col + (int64_t)jn * sstride);
    else win[WN - 1] = PT{};
  }
}

template <int K, int SIDE>
static hipError_t launch_project_k(const uint8_t* src, int64_t pitch, int64_t sstride, int S, int H, int W,
                                   const uint8_t* excl, uint8_t* dst, int64_t dpitch, int64_t dstride,
                                   hipStream_t st) {
  const bool vec = (W % 16 == 0) && (pitch % 16 == 0) && (sstride % 16 == 0) && (dpitch % 16 == 0) &&
                   (dstride % 16 == 0) && (((uintptr_t)src) % 16 == 0) && (((uintptr_t)dst) % 16 == 0);
  if (vec) {
    const long long nthr = (long long)H * (W / 16);
    k_project<K, 16, SIDE><<<(unsigned)((nthr + 255) / 256), 256, 0, st>>>(src, pitch, sstride, S, H, W, excl, dst,
                                                                            dpitch, dstride);
  } else {
    const long long nthr = (long long)H * W;
    k_project<K, 1, SIDE><<<(unsigned)((nthr + 255) / 256), 256, 0, st>>>(src, pitch, sstride, S, H, W, excl, dst,
                                                                           dpitch, dstride);
  }
  return hipGetLastError();
}

hipError_t launch_project(const uint8_t* src, int64_t pitch, int64_t sstride, int S, int H, int W,
                          const uint8_t* excl, int k, uint8_t* dst, int64_t dpitch, int64_t dstride,
                          hipStream_t st, KernelTimer* kt, int side) {
  if (kt) kt->begin(side == 0 ? "k_project" : (side < 0 ? "k_project_left" : "k_project_right"), k, st);
  hipError_t e;
  if (side == 0)
    e = launch_project_sel<0>(src, pitch, sstride, S, H, W, excl, k, dst, dpitch, dstride, st);
  else if (side < 0)
    e = launch_project_sel<-1>(src, pitch, sstride, S, H, W, excl, k, dst, dpitch, dstride, st);
  else
    e = launch_project_sel<1>(src, pitch, sstride, S, H, W, excl, k, dst, dpitch, dstride, st);
  if (kt) kt->end(st);
  return e;
}

template <int SIDE>
hipError_t launch_project_sel(const uint8_t* src, int64_t pitch, int64_t sstride, int S, int H, int W,
                              const uint8_t* excl, int k, uint8_t* dst, int64_t dpitch, int64_t dstride,
                              hipStream_t st) {
  switch (k) {
    case 1: return launch_project_k<1, SIDE>(src, pitch, sstride, S, H, W, excl, dst, dpitch, dstride, st);
    case 2: return launch_project_k<2, SIDE>(src, pitch, sstride, S, H, W, excl, dst, dpitch, dstride, st);
    case 3: return launch_project_k<3, SIDE>(src, pitch, sstride, S, H, W, excl, dst, dpitch, dstride, st);
    case 4: return launch_project_k<4, SIDE>(src, pitch, sstride, S, H, W, excl, dst, dpitch, dstride, st);
    case 5: return launch_project_k<5, SIDE>(src, pitch, sstride, S, H, W, excl, dst, dpitch, dstride, st);
    case 6: return launch_project_k<6, SIDE>(src, pitch, sstride, S, H, W, excl, dst, dpitch, dstride, st);
    case 7: return launch_project_k<7, SIDE>(src, pitch, sstride, S, H, W, excl, dst, dpitch, dstride, st);
    case 8: return launch_project_k<8, SIDE>(src, pitch, sstride, S, H, W, excl, dst, dpitch, dstride, st);
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------- refinement step
__global__ void __launch_bounds__(256) k_refine(int P, const swift_match* __restrict__ rec,
                                                const float* __restrict__ jac, float* __restrict__ th, int mode,
                                                float max_step, float* __restrict__ step_out) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= P) return;
  const swift_match r = rec[i];
  const int n = r.n > 0 ? r.n : 1;
  const int sx = r.ix >= n / 2 ? r.ix - n : r.ix, sy = r.iy >= n / 2 ? r.iy - n : r.iy;
  float dx = -r.dx, dy = -r.dy;  // centroid step
  float limit = max_step;
  if (mode == SWIFT_REFINE_NEWTON && jac && abs(sx) <= 1 && abs(sy) <= 1 && !(r.status & SWIFT_ST_DEGENERATE)) {
    // Newton on the centroid within the cell of the integer peak s:
    // d = s + J (t - t* - s)  =>  t <- t - (s + J^-1 (d - s)), J = d d / d t
    const float* q = jac + (size_t)i * 12;
    const double j00 = q[2], j01 = q[5], j10 = q[8], j11 = q[11];
    const double det = j00 * j11 - j01 * j10;
    if (det > 1e-6) {
      const double ex = (double)r.dx - sx, ey = (double)r.dy - sy;
      const double ox = (j11 * ex - j01 * ey) / det, oy = (-j10 * ex + j00 * ey) / det;  // offset within the cell
      // away from the origin the linear model must place t inside the peak's cell
      if ((sx == 0 && sy == 0) || (fabs(ox) <= 0.6 && fabs(oy) <= 0.6)) {
        dx = (float)(-(sx + ox));
        dy = (float)(-(sy + oy));
        limit = max_step + sqrtf((float)(sx * sx + sy * sy));  // never cut the whole-pixel part
      }
    }
  }
  float len = sqrtf(dx * dx + dy * dy);
  if (!(len <= limit)) {  // also catches NaN
    const float sc = (len > 0.0f && len == len) ? limit / len : 0.0f;
    dx *= sc;
    dy *= sc;
    len = (len == len) ? limit : 0.0f;
  }
  th[(size_t)i * 8 + 4] += dx;
  th[(size_t)i * 8 + 7] += dy;
  if (step_out) step_out[i] = len;
}

hipError_t launch_refine(int P, const swift_match* rec, const float* jac, float* th, int mode, float max_step,
                         float* step_out, hipStream_t st) {
  if (P > 0) k_refine<<<(P + 255) / 256, 256, 0, st>>>(P, rec, jac, th, mode, max_step, step_out);
  return hipGetLastError();
}

// ---------------------------------------------------------------- x2 pyramid
// dst(x, y) = (src(2x,2y) + src(2x+1,2y) + src(2x,2y+1) + src(2x+1,2y+1) + 2) >> 2
__global__ void __launch_bounds__(256) k_pyramid(const uint8_t* __restrict__ src, int64_t spitch,
                                                 uint8_t* __restrict__ dst, int64_t dpitch, int dw, int dh) {
  const long long gid = (long long)blockIdx.x * 256 + threadIdx.x;
  if (gid >= (long long)dw * dh) return;
  const int y = (int)(gid / dw), x = (int)(gid % dw);
  const uint8_t* r0 = src + (int64_t)(2 * y) * spitch + 2 * x;
  const uint8_t* r1 = r0 + spitch;
  const uint32_t s = (uint32_t)r0[0] + r0[1] + r1[0] + r1[1];
  dst[(int64_t)y * dpitch + x] = (uint8_t)((s + 2u) >> 2);
}

hipError_t launch_pyramid(const uint8_t* src, int64_t spitch, int sw, int sh, uint8_t* dst, int64_t dpitch,
                          int dw, int dh, hipStream_t st) {
  (void)sw;
  (void)sh;
  const long long n = (long long)dw * dh;
  if (n > 0) k_pyramid<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(src, spitch, dst, dpitch, dw, dh);
  return hipGetLastError();
}

// ---------------------------------------------------------------- jump repair blend
// Affines of the failed span [a, b]: aff[s] = (1 - w) left[s] + w right[s]
// per entry, w = 3 t^2 - 2 t^3 (the cubic Bezier with control values 0, 0,
// 1, 1), t = (s - a + 1) / (b - a + 2).  One thread per entry.
__global__ void __launch_bounds__(64) k_blend_span(int a, int b, const double* __restrict__ left,
                                                   const double* __restrict__ right, double* __restrict__ aff) {
  const int i = blockIdx.x * 64 + threadIdx.x;
  if (i >= 6 * (b - a + 1)) return;
  const int s = a + i / 6, e = i % 6;
  const double t = (double)(s - a + 1) / (double)(b - a + 2);
  const double w = 3.0 * t * t - 2.0 * t * t * t;
  aff[6 * (size_t)s + e] = (1.0 - w) * left[6 * (size_t)s + e] + w * right[6 * (size_t)s + e];
}

hipError_t launch_blend_span(int a, int b, const double* left, const double* right, double* aff, hipStream_t st) {
  const int n = 6 * (b - a + 1);
  if (n > 0) k_blend_span<<<(n + 63) / 64, 64, 0, st>>>(a, b, left, right, aff);
  return hipGetLastError();
}

// Break join: D = A_j^-1 L_j (aligned-frame correction from section j's fit
// against its left one-sided model); out[s] = in[s] o D for s >= j, in[s]
// otherwise.  Out of place: every thread reads A_j from `in`.
__global__ void __launch_bounds__(64) k_join_break(int S, int j, const double* __restrict__ in,
                                                   const double* __restrict__ left, double* __restrict__ out) {
  const int s = blockIdx.x * 64 + threadIdx.x;
  if (s >= S) return;
  const double* A = in + 6 * (size_t)s;
  double* O = out + 6 * (size_t)s;
  if (s < j) {
    for (int e = 0; e < 6; ++e) O[e] = A[e];
    return;
  }
  const double* Aj = in + 6 * (size_t)j;
  const double* Lj = left + 6 * (size_t)j;
  // A_j^-1 = [M^-1, -M^-1 t]
  const double det = Aj[0] * Aj[4] - Aj[1] * Aj[3];
  const double i00 = Aj[4] / det, i01 = -Aj[1] / det, i10 = -Aj[3] / det, i11 = Aj[0] / det;
  const double it0 = -(i00 * Aj[2] + i01 * Aj[5]), it1 = -(i10 * Aj[2] + i11 * Aj[5]);
  // D = A_j^-1 L_j
  const double d00 = i00 * Lj[0] + i01 * Lj[3], d01 = i00 * Lj[1] + i01 * Lj[4];
  const double d10 = i10 * Lj[0] + i11 * Lj[3], d11 = i10 * Lj[1] + i11 * Lj[4];
  const double dt0 = i00 * Lj[2] + i01 * Lj[5] + it0, dt1 = i10 * Lj[2] + i11 * Lj[5] + it1;
  // out = A o D
  const double o00 = A[0] * d00 + A[1] * d10, o01 = A[0] * d01 + A[1] * d11;
  const double o10 = A[3] * d00 + A[4] * d10, o11 = A[3] * d01 + A[4] * d11;
  const double ot0 = A[0] * dt0 + A[1] * dt1 + A[2], ot1 = A[3] * dt0 + A[4] * dt1 + A[5];
  O[0] = o00;
  O[1] = o01;
  O[2] = ot0;
  O[3] = o10;
  O[4] = o11;
  O[5] = ot1;
}

hipError_t launch_join_break(int S, int j, const double* in, const double* left, double* out, hipStream_t st) {
  if (S > 0) k_join_break<<<(S + 63) / 64, 64, 0, st>>>(S, j, in, left, out);
  return hipGetLastError();
}

// ---------------------------------------------------------------- search with an SNR stop
// The n active windows idx[i] (of P) were matched at candidate `cand`
// (records recs[i]): each keeps the higher-SNR of its kept record and the
// new one (the earlier candidate on equal SNR) and is done once the kept SNR
// reaches `accept`.  Window indices outside [0, P), and windows already
// done (a caller matching several candidates ahead), are left alone.
__global__ void __launch_bounds__(256) k_search_keep(int P, int n, const int32_t* __restrict__ idx,
                                                     const swift_match* __restrict__ recs, int cand, float accept,
                                                     swift_match* __restrict__ best, int32_t* __restrict__ best_cand,
                                                     uint8_t* __restrict__ done) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int w = idx[i];
  if (w < 0 || w >= P || done[w]) return;
  const swift_match r = recs[i];
  if (best_cand[w] < 0 || r.snr > best[w].snr) {
    best[w] = r;
    best_cand[w] = cand;
  }
  if (best[w].snr >= accept) done[w] = 1;
}

hipError_t launch_search_keep(int P, int n, const int32_t* idx, const swift_match* recs, int cand, float accept,
                              swift_match* best, int32_t* best_cand, uint8_t* done, hipStream_t st) {
  if (n > 0) k_search_keep<<<(n + 255) / 256, 256, 0, st>>>(P, n, idx, recs, cand, accept, best, best_cand, done);
  return hipGetLastError();
}

// Next round of the search: the windows not yet done, in ascending order
// (a sorted batch stays sorted), gathered with window A moved by (ox, oy).
// One workgroup walks the windows 1024 at a time; a wave's ballot gives each
// searching window its place within the wave, and the per-wave counts in LDS
// give the wave's base.  count receives the number gathered.
__global__ void __launch_bounds__(1024) k_search_next(int P, const uint8_t* __restrict__ done, float ox, float oy,
                                                      const int32_t* __restrict__ img_a,
                                                      const int32_t* __restrict__ img_b,
                                                      const float* __restrict__ theta_a,
                                                      const float* __restrict__ theta_b, int32_t* __restrict__ idx,
                                                      int32_t* __restrict__ ia, int32_t* __restrict__ ib,
                                                      float* __restrict__ ta, float* __restrict__ tb,
                                                      int32_t* __restrict__ count) {
  __shared__ int wsum[16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  int base = 0;
  for (int c0 = 0; c0 < P; c0 += 1024) {
    const int w = c0 + (int)threadIdx.x;
    const bool f = w < P && done[w] == 0;
    const unsigned long long b = __ballot(f);
    const int pre = __popcll(b & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wid] = __popcll(b);
    __syncthreads();
    int off = 0, tot = 0;
    for (int i = 0; i < 16; ++i) {
      off += i < wid ? wsum[i] : 0;
      tot += wsum[i];
    }
    if (f) {
      const int o = base + off + pre;
      idx[o] = w;
      ia[o] = img_a[w];
      ib[o] = img_b[w];
      for (int k = 0; k < 8; ++k) {
        float va = theta_a[(size_t)w * 8 + k];
        if (k == 4) va += ox;
        if (k == 7) va += oy;
        ta[(size_t)o * 8 + k] = va;
        tb[(size_t)o * 8 + k] = theta_b[(size_t)w * 8 + k];
      }
    }
    base += tot;
    __syncthreads();  // wsum is rewritten by the next chunk
  }
  if (threadIdx.x == 0) *count = base;
}

hipError_t launch_search_next(int P, const uint8_t* done, float ox, float oy, const int32_t* img_a,
                              const int32_t* img_b, const float* theta_a, const float* theta_b, int32_t* idx,
                              int32_t* ia, int32_t* ib, float* ta, float* tb, int32_t* count, hipStream_t st) {
  k_search_next<<<1, 1024, 0, st>>>(P, done, ox, oy, img_a, img_b, theta_a, theta_b, idx, ia, ib, ta, tb, count);
  return hipGetLastError();
}

}  // namespace swift
