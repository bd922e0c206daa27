// Device helpers shared by the matching and scoring kernels.
#pragma once
#include <float.h>
#include <limits.h>
#include <math.h>

#include "swift_fft.hpp"
#include "swift_internal.hpp"

namespace swift {

// Pointers into the images come from the device image table, so the compiler
// cannot prove they are global memory; this cast lets it use global (not flat)
// loads.
template <typename T>
using gptr = const __attribute__((address_space(1))) T*;
template <typename T>
__device__ __forceinline__ gptr<T> to_global(const void* p) {
  return (gptr<T>)p;
}

__device__ __forceinline__ float taper_at(int i, int n, int L) {
  if (L <= 0) return 1.0f;
  const int m = i < n - 1 - i ? i : n - 1 - i;
  if (m >= L) return 1.0f;
  return 0.5f * (1.0f - cospif(((float)m + 0.5f) / (float)L));
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Wave-wide FP32 sum, all in registers: DPP within rows of 16 lanes (every
// lane of a row then holds the row's sum), then the row broadcasts of the
// wave64 DPP controls fold rows 0..2 into row 3; lane 63 holds the total,
// returned to every lane.
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROWS, 0xF, false));
}
__device__ __forceinline__ float wave_sum_f32(float v) {
  v += dpp_f32<0xB1>(v);        // quad_perm [1,0,3,2]
  v += dpp_f32<0x4E>(v);        // quad_perm [2,3,0,1]
  v += dpp_f32<0x124>(v);       // row_ror:4
  v += dpp_f32<0x128>(v);       // row_ror:8
  v += dpp_f32<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v += dpp_f32<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Inclusive prefix sum over the 64 lanes of a wave: shifts by 1, 2, 4, 8
// within each row of 16 lanes (lanes with no source add 0), then row 0's
// total into row 1 and row 2's into row 3, then lanes 0..31's total into rows
// 2 and 3.
__device__ __forceinline__ float wave_incl_scan_f32(float v) {
  v += dpp_f32<0x111>(v);
  v += dpp_f32<0x112>(v);
  v += dpp_f32<0x114>(v);
  v += dpp_f32<0x118>(v);
  v += dpp_f32<0x142, 0xA>(v);
  v += dpp_f32<0x143, 0xC>(v);
  return v;
}

// Layout of the row spectra exchanged between the forward row pass and the
// column pass (and of the column pass's output for the inverse row pass):
// tiles of 8 rows, Z[pair][y / 8][kx][y % 8].  A row block of 8 rows writes
// one contiguous 8 N-element region; a column is read as runs of 8 elements.
template <int N>
__device__ __forceinline__ size_t ztile(int kx, int y) {
  return (size_t)(y >> 3) * (8 * N) + (size_t)kx * 8 + (y & 7);
}

// Splits one bin of the packed spectrum z = a'T + i b'T into the normalised,
// mean-free window spectra: zp = Z(k), zm = conj Z(-k), tk = tau(ky) tau(kx);
// F_A = (zp + zm) / 2 - mA tk and F_B = (zp - zm) / (2i) - mB tk, each scaled
// by its 1 / ||w|| (sA, sB), so products of them stay in FP32 range.
__device__ __forceinline__ void split_bin(float2 zp, float2 zm, float2 tk, const PairStat& ps, float2& fa,
                                          float2& fb) {
  const float ha = 0.5f * ps.sA, hb = 0.5f * ps.sB;
  fa = csub(cscale(cadd(zp, zm), ha), cscale(tk, ps.mA * ps.sA));
  const float2 dd = csub(zp, zm);
  fb = csub(make_float2(hb * dd.y, -hb * dd.x), cscale(tk, ps.mB * ps.sB));
}

// Pair statistics from the window sums of the whole pair (s as in RowPart,
// summed over the row slices): taper-weighted means m = sum a'T / (sum T)^2,
// energies ||w||^2 = sum (a'T)^2 - 2 m sum a'T^2 + m^2 (sum T^2)^2, the
// degeneracy test and the whitening scales.
__device__ inline PairStat make_pair_stat(const double (&s)[6], bool clamped, const TaperInfo& ti, float oA, float oB,
                                          int n, bool pearson, float p) {
  const double sT = ti.sum_t * ti.sum_t, sT2 = ti.sum_t2 * ti.sum_t2;
  const double mA = s[0] / sT, mB = s[3] / sT;
  const double wA = s[1] - 2.0 * mA * s[2] + mA * mA * sT2;
  const double wB = s[4] - 2.0 * mB * s[5] + mB * mB * sT2;
  PairStat ps;
  ps.mA = (float)mA;
  ps.mB = (float)mB;
  ps.oA = oA;
  ps.oB = oB;
  ps.swA = (float)fmax(wA, 0.0);
  ps.swB = (float)fmax(wB, 0.0);
  ps.pad[0] = ps.pad[1] = 0;
  // degenerate: a window's weighted variance is at most kDegenerateRel of
  // its energy about the offset (samples equal up to rounding; a constant
  // window has all sums exactly 0)
  const bool degA = !(wA > kDegenerateRel * s[1]), degB = !(wB > kDegenerateRel * s[4]);
  ps.flags = (clamped ? 4 : 0) | ((degA || degB) ? 1 : 0);
  const double inv_m = 1.0 / ((double)n * (double)n);
  if (pearson) {
    // the template carries the mean (its spectrum has no DC), so window B is
    // used as gathered; only a constant template is degenerate (a constant
    // patch of B gets a zero coefficient per placement).  No whitening (p =
    // 0): the spectra are used unscaled.
    ps.mB = 0.0f;
    ps.flags = (clamped ? 4 : 0) | (degA ? 1 : 0);
  }
  if (ps.flags & 1) {
    ps.sA = ps.sB = 0.0f;
    ps.kw = 0.0f;
  } else if (pearson) {
    ps.sA = ps.sB = 1.0f;
    ps.kw = (float)inv_m;
  } else {
    ps.sA = (float)(1.0 / sqrt(wA));
    ps.sB = (float)(1.0 / sqrt(wB));
    ps.kw = (float)(exp(0.5 * (1.0 - (double)p) * (log(wA) + log(wB))) * inv_m);
  }
  return ps;
}

// Whitening of one bin.
// zp = Z(k), zm = conj Z(-k) of the packed spectrum z = a'T + i b'T, tk =
// tau(ky) tau(kx).  Splits F_A = (zp + zm) / 2, F_B = (zp - zm) / (2i),
// removes the weighted means (F -= m tk), and scales both by 1 / ||w||, so the
// normalised cross power X^ = conj(F_A^) F_B^ has |X^| <= N^2 whatever the
// input scale.  With X = X^ ||w_A|| ||w_B|| and eps = eps_rel ||w_A|| ||w_B||,
//   C = X (|X|^2 + eps^2)^(-p/2) / N^2 = X^ (|X^|^2 + eps_rel^2)^(-p/2) kw,
// kw = (||w_A|| ||w_B||)^(1-p) / N^2.  The DC bin (and a degenerate pair) gives 0.
__device__ __forceinline__ float2 whiten_bin(float2 zp, float2 zm, float2 tk, const PairStat& ps, float p,
                                             float eps_rel, bool dc) {
  float2 fa, fb;
  split_bin(zp, zm, tk, ps, fa, fb);
  const float2 X = make_float2(fa.x * fb.x + fa.y * fb.y, fa.x * fb.y - fa.y * fb.x);
  const float d = fmaf(X.x, X.x, fmaf(X.y, X.y, eps_rel * eps_rel));
  float gs;
  if (p == 0.0f) gs = 1.0f;
  else if (!(d > 0.0f)) gs = 0.0f;
  else if (p == 1.0f) gs = __builtin_amdgcn_rsqf(d);
  else gs = __builtin_amdgcn_exp2f(-0.5f * p * __builtin_amdgcn_logf(d));
  gs *= ps.kw;
  if (dc) gs = 0.0f;
  return cscale(X, gs);
}

struct Top2 {
  float m1;
  int i1;
  float m2;
};

__device__ __forceinline__ void top2_push(Top2& a, float v, int i) {
  if (v > a.m1 || (v == a.m1 && i < a.i1)) {
    a.m2 = a.m1;
    a.m1 = v;
    a.i1 = i;
  } else if (v > a.m2) {
    a.m2 = v;
  }
}

// For values visited in increasing index order within a lane: a strict >
// already keeps the first maximum.
__device__ __forceinline__ void top2_push_ordered(Top2& a, float v, int i) {
  const bool c1 = v > a.m1;
  a.m2 = c1 ? a.m1 : fmaxf(a.m2, v);
  a.i1 = c1 ? i : a.i1;
  a.m1 = c1 ? v : a.m1;
}

__device__ __forceinline__ Top2 top2_merge(Top2 a, Top2 b) {
  const bool bw = (b.m1 > a.m1) || (b.m1 == a.m1 && b.i1 < a.i1);
  Top2 w = bw ? b : a, l = bw ? a : b;
  Top2 r;
  r.m1 = w.m1;
  r.i1 = w.i1;
  r.m2 = fmaxf(l.m1, fmaxf(a.m2, b.m2));
  return r;
}

__device__ __forceinline__ Top2 wave_top2(Top2 a) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    Top2 o;
    o.m1 = __shfl_xor(a.m1, off);
    o.i1 = __shfl_xor(a.i1, off);
    o.m2 = __shfl_xor(a.m2, off);
    a = top2_merge(a, o);
  }
  return a;
}

// Match record from the reduced surface statistics and the 3x3 neighbourhood
// nb[dy+1][dx+1] of the peak (nb[1][1] is replaced by the peak value).
// Z-score over the whole surface (population std, FP64); centroid weights
// max(c - mean, 0); integer shifts wrapped to [-n/2, n/2).
// count: number of surface entries the sums cover (n^2 unless given).
__device__ inline swift_match make_record(int n, Top2 tp, double sum, double sq, float (*nb)[3], int flags,
                                          double count = 0.0) {
  const int flat = (tp.i1 >= 0 && tp.i1 < n * n) ? tp.i1 : 0;
  const int iy = flat / n, ix = flat % n;
  const double M = count > 0.0 ? count : (double)n * (double)n;
  const double mu = sum / M;
  const double var = fmax(sq / M - mu * mu, 0.0);
  const double sd = sqrt(var);
  swift_match rec;
  rec.ix = ix;
  rec.iy = iy;
  rec.n = n;
  rec.peak = tp.m1;
  rec.mean = mu;
  rec.std = sd;
  int st = flags;
  if (tp.m1 - tp.m2 <= kNearTieRel * fabsf(tp.m1)) st |= SWIFT_ST_NEAR_TIE;
  if (sd > 0.0) {
    rec.snr = (float)(((double)tp.m1 - mu) / sd);
  } else {
    rec.snr = 0.0f;
    st |= SWIFT_ST_DEGENERATE;
  }
  nb[1][1] = tp.m1;
  double sw = 0.0, swx = 0.0, swy = 0.0;
  for (int dy = -1; dy <= 1; ++dy)
    for (int dx = -1; dx <= 1; ++dx) {
      const double wv = fmax((double)nb[dy + 1][dx + 1] - mu, 0.0);
      sw += wv;
      swx += wv * dx;
      swy += wv * dy;
    }
  const int sx = ix >= n / 2 ? ix - n : ix;
  const int sy = iy >= n / 2 ? iy - n : iy;
  rec.dx = (float)(sx + (sw > 0.0 ? swx / sw : 0.0));
  rec.dy = (float)(sy + (sw > 0.0 ? swy / sw : 0.0));
  rec.status = st;
  rec.hxx = nb[1][0] - 2.0f * nb[1][1] + nb[1][2];
  rec.hyy = nb[0][1] - 2.0f * nb[1][1] + nb[2][1];
  rec.hxy = 0.25f * (nb[2][2] - nb[0][2] - nb[2][0] + nb[0][0]);
  rec.reserved = 0;
  return rec;
}

}  // namespace swift
