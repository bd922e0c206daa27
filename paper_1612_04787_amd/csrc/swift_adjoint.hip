// Adjoint of the whitened match: gradient of J = g_peak c[s*] + g_snr SNR with
// respect to the six affine entries of both windows, the integer peak s* held
// fixed.  (Not in the paper; the chain rule through the plain definition.)
//
// Notation (full N x N spectrum, M = N^2, k != 0):
//   X = conj(F_A) F_B,  r = |X|^2,  d = r + eps^2,  h = d^(-p/2),
//   h' = dh/dd = -(p/2) h / d,  c = IDFT(X h) (1/M scaled).
// Surface cotangent: G_c = alpha delta(s*) + beta + gamma (c - mean) with
//   alpha = g_peak + g_snr / sigma, gamma = -g_snr SNR / (M sigma^2),
// so its spectrum needs no transform: G_C = (alpha e^{-2 pi i k.s*/N} + gamma X h) / M.
// Then (complex gradients G = dJ/dRe + i dJ/dIm):
//   G_X = G_C (h + r h') + conj(G_C) X^2 h',   dJ/d(eps^2) = sum Re(conj(G_C) X h'),
//   G_FA = conj(G_X) F_B,  G_FB = G_X F_A.
// Both are Hermitian, so one complex inverse 2-D FFT of Q = G_FA + i G_FB gives
// G_wA (real part) and G_wB (imaginary part), unnormalised.  With
// lambda_A = dJ/d(eps^2) 2 eps_rel^2 ||w_B||^2 (eps^2 depends on ||w||), the mean
// removal and taper give G_a = T (G_w + lambda w) - (T / sum T) sum T (G_w + lambda w),
// and the bilinear gather dtheta = sum_px G_a D with
//   D = (a_x u, a_x v, a_x, a_y u, a_y v, a_y)   (a_x, a_y: bilinear partials).
// Expanding, dtheta = P1 + lambda P3 - (Q + lambda R) / sum T * P2 where
//   P1 = sum T G_w D, P2 = sum T D, P3 = sum T w D, Q = sum T G_w, R = sum T w
// are plain per-pixel sums, so the row stage needs no second pass.
//
// The column stage works with the normalised spectra F^ = F / ||w|| of the
// forward pass (split_bin), X^ = X s with s = 1 / (||w_A|| ||w_B||), so no
// FP32 square overflows: h = s^p h^, h' = -(p/2) s^(p+2) h^ / d^ with
// d^ = |X^|^2 + eps_rel^2, hence G_X = s^p [G_C (h^ + r^ h^') + conj(G_C) X^^2 h^']
// (h^' = -(p/2) h^ / d^), dJ/d(eps^2) = s^(p+1) sum Re(conj(G_C) X^ h^') and
// X h = s^(p-1) X^ h^ (= kw N^2 X^ h^).
//
// Kernels per window size: k_bwd_col (column stage), k_bwd_row (inverse row
// FFTs + gather recomputation + sums), k_bwd_fin (per pair).
//
// Centroid-Jacobian mode (CJ): the objectives are the two components of the
// centroid shift d = s* + sum_delta w_delta delta / sum w (w = max(c - mean, 0)
// on the 3 x 3 box), whose surface cotangent is nine weighted deltas,
//   d(dx)/dc(s* + delta) = (delta_x - (dx - sx)) / sum w   (w > 0),
// (the mean's share is uniform and vanishes with the DC bin), so again
// G_C = e^{-2 pi i k.s*/N} / M sum_delta omega_delta e^{-2 pi i k.delta/N}.
// Only window A is differentiated: G_FA of the x objective goes to the real
// channel and that of the y objective to the imaginary channel of the one
// inverse 2-D FFT, giving d(dx, dy) / d theta_A in a single pass.
#include "swift_dev.hpp"
#include "swift_tile.hpp"

namespace swift {

// ---------------------------------------------------------------- column stage
// One FFT group per column pair (kx = w and its mirror N - w): the group
// reads both saved forward spectra, forms Q(., w) = G_FA + i G_FB and, through
// its own two LDS slots, Q(., N - w), and inverse-transforms both columns.
template <int N>
constexpr int bwd_col_blocks() {
  return (N / 2 + 1 + 256 / FftCfg<N>::T - 1) / (256 / FftCfg<N>::T);
}

template <int N, bool CJ>
__global__ void __launch_bounds__(256) k_bwd_col(BwdArgs a) {
  using C = FftCfg<N>;
  constexpr int T = C::T, E = C::E, G = 256 / T;
  constexpr int NI = N / 2 + 1, NW = bwd_col_blocks<N>();
  constexpr int SL = fft_scratch<N>();
  __shared__ float2 lds[2 * G * SL];
  __shared__ double red[4][kDpart];

  const int pair = blockIdx.x / NW, wg = blockIdx.x % NW;
  const int tid = threadIdx.x, c = tid / T, t = tid % T;
  const int w = wg * G + c;
  const bool valid = w < NI;
  const int wm = (N - w) & (N - 1);  // mirror column
  float2* slotA = lds + (2 * c) * SL;
  float2* slotB = lds + (2 * c + 1) * SL;
  float2 v[E], u[E];
  if (valid) {
    const float2* src = a.Zf + (size_t)pair * N * N;
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = src[(size_t)w * N + t + e * T];
#pragma unroll
    for (int e = 0; e < E; ++e) u[e] = src[(size_t)wm * N + t + e * T];
#pragma unroll
    for (int e = 0; e < E; ++e) slotB[lidx(t + e * T)] = u[e];
  }
  wave_lds_sync();

  float dj = 0.0f, dj1 = 0.0f, hxx = 0.0f, hyy = 0.0f, hxy = 0.0f;
  if (valid) {
    const PairStat ps = a.ps[pair];
    const swift_match rec = a.rec[pair];
    const float gp = a.g_peak ? a.g_peak[pair] : 0.0f;
    const float gsn = a.g_snr ? a.g_snr[pair] : 0.0f;
    float alpha = gp, gamma = 0.0f;
    if (rec.std > 0.0) {
      const double snr = ((double)rec.peak - rec.mean) / rec.std;
      alpha = (float)((double)gp + (double)gsn / rec.std);
      gamma = (float)(-(double)gsn * snr / ((double)N * N * rec.std * rec.std));
    }
    bool zero_all = (ps.flags & 1) != 0;
    // centroid weights (CJ): omega_x, omega_y on the 3 x 3 box, from the saved values
    float omx[9], omy[9];
    float2 rxw[3], ryw[3];
    if constexpr (CJ) {
      const float* q = a.nb + (size_t)pair * 9;
      double sw = 0.0, swx = 0.0, swy = 0.0;
      for (int j = 0; j < 9; ++j) {
        const double wv = fmax((double)q[j] - rec.mean, 0.0);
        sw += wv;
        swx += wv * (double)(j % 3 - 1);
        swy += wv * (double)(j / 3 - 1);
      }
      const double fxc = sw > 0.0 ? swx / sw : 0.0, fyc = sw > 0.0 ? swy / sw : 0.0;
#pragma unroll
      for (int j = 0; j < 9; ++j) {
        const bool on = sw > 0.0 && (double)q[j] - rec.mean > 0.0;
        omx[j] = on ? (float)(((double)(j % 3 - 1) - fxc) / sw) : 0.0f;
        omy[j] = on ? (float)(((double)(j / 3 - 1) - fyc) / sw) : 0.0f;
      }
      if (!(sw > 0.0)) zero_all = true;
      const float2 ex = a.tw[w * (1024 / N)], exc = cconj(ex);
      const float im_ = 1.0f / (float)(N * N);
#pragma unroll
      for (int r3 = 0; r3 < 3; ++r3) {
        rxw[r3] = cscale(cadd(cadd(cscale(exc, omx[3 * r3]), make_float2(omx[3 * r3 + 1], 0.f)),
                              cscale(ex, omx[3 * r3 + 2])), im_);
        ryw[r3] = cscale(cadd(cadd(cscale(exc, omy[3 * r3]), make_float2(omy[3 * r3 + 1], 0.f)),
                              cscale(ex, omy[3 * r3 + 2])), im_);
      }
      // S(ky) = e_y^-1 rw[0] + rw[1] + e_y rw[2] with e_y = (cy, sy):
      //       = rw[1] + cy (rw[0] + rw[2]) + sy i (rw[2] - rw[0])
      const float2 dx2 = csub(rxw[2], rxw[0]), dy2 = csub(ryw[2], ryw[0]);
      rxw[0] = cadd(rxw[0], rxw[2]);
      ryw[0] = cadd(ryw[0], ryw[2]);
      rxw[2] = make_float2(-dx2.y, dx2.x);
      ryw[2] = make_float2(-dy2.y, dy2.x);
    }
    const float p = a.p, hp2 = -0.5f * p;
    const float inv_m = 1.0f / (float)(N * N);
    const float e2 = a.eps_rel * a.eps_rel;
    // per-pair scales of the normalised spectra: X h = kwm X^ h^, and
    // G_FA = (s^p ||w_B||) conj(G_X^) F_B^, G_FB = (s^p ||w_A||) G_X^ F_A^
    const float kwm = ps.kw * (float)(N * N);
    float sca = 0.0f, scb = 0.0f;
    if (!zero_all && ps.sA > 0.0f && ps.sB > 0.0f) {
      const double sp = pow((double)ps.sA * (double)ps.sB, (double)p);
      sca = (float)(sp / (double)ps.sB);
      scb = (float)(sp / (double)ps.sA);
    }
    const float mw = (w == 0 || w == N / 2) ? 1.0f : 2.0f;  // column w and its mirror N - w
    const float2 tauw = a.tau[w];
    // signed frequency of the column (Nyquist: squared terms only)
    const float fw = (float)w, fwm = (w == N / 2) ? 0.0f : (float)w;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int ky = t + e * T;
      float2 fa, fb;  // F_A^, F_B^
      split_bin(v[e], cconj(slotB[lidx((N - ky) & (N - 1))]), cmul(a.tau[ky], tauw), ps, fa, fb);
      const float2 X = make_float2(fa.x * fb.x + fa.y * fb.y, fa.x * fb.y - fa.y * fb.x);  // X^
      const float r = X.x * X.x + X.y * X.y;
      const float d = r + e2;
      float h, hd;  // h^ and h^' = dh^/dd^
      if (p == 0.0f) {
        h = 1.0f;
        hd = 0.0f;
      } else if (!(d > 0.0f)) {
        h = 0.0f;
        hd = 0.0f;
      } else {
        h = (p == 1.0f) ? __builtin_amdgcn_rsqf(d) : __builtin_amdgcn_exp2f(hp2 * __builtin_amdgcn_logf(d));
        hd = hp2 * h * __builtin_amdgcn_rcpf(d);
      }
      // e^{-2 pi i (ky iy + w ix) / N} from the W_1024 table
      const int m = (ky * rec.iy + w * rec.ix) & (N - 1);
      const float2 ph = a.tw[m * (1024 / N)];
      // surface Hessian sums: Re(X h e^{+i phi}) times the frequency products
      if (!CJ && !zero_all && !(ky == 0 && w == 0)) {
        const float2 cc = cmul(cscale(X, h * kwm), cconj(ph));
        const float fy = (ky < N / 2) ? (float)ky : (float)(ky - N);
        const float fym = (ky == N / 2) ? 0.0f : fy;
        hxx += mw * cc.x * fw * fw;
        hyy += mw * cc.x * fy * fy;
        hxy += mw * cc.x * fwm * fym;
      }
      // G_X = G_C (h + r h') + conj(G_C) X^2 h'
      const float hr = fmaf(r, hd, h);
      const float2 x2h = cscale(cmul(X, X), hd);
      const float2 xh = cscale(X, mw * hd);
      const bool zb = zero_all || (ky == 0 && w == 0);
      float2 gfa, gfb;
      if constexpr (!CJ) {
        float2 gc = cscale(cadd(cscale(ph, alpha), cscale(X, gamma * h * kwm)), inv_m);
        if (zb) gc = make_float2(0.0f, 0.0f);
        const float2 gx = cadd(cscale(gc, hr), cmul(cconj(gc), x2h));
        dj = fmaf(gc.x, xh.x, fmaf(gc.y, xh.y, dj));
        gfa = cscale(cmul(cconj(gx), fb), sca);
        gfb = cscale(cmul(gx, fa), scb);
      } else {
        // 3 x 3 sums S = sum omega e_x^dx e_y^dy / M with e = e^{-2 pi i k/N};
        // the x part (rows of the box summed over dx) is the same for the whole
        // column and is folded into rw so that S = rw[1] + cy rw[0] + sy rw[2]
        const float2 ey = a.tw[ky * (1024 / N)];
        const float2 sx = make_float2(fmaf(ey.y, rxw[2].x, fmaf(ey.x, rxw[0].x, rxw[1].x)),
                                      fmaf(ey.y, rxw[2].y, fmaf(ey.x, rxw[0].y, rxw[1].y)));
        const float2 sy = make_float2(fmaf(ey.y, ryw[2].x, fmaf(ey.x, ryw[0].x, ryw[1].x)),
                                      fmaf(ey.y, ryw[2].y, fmaf(ey.x, ryw[0].y, ryw[1].y)));
        float2 gcx = cmul(ph, sx), gcy = cmul(ph, sy);
        if (zb) gcx = gcy = make_float2(0.0f, 0.0f);
        const float2 gxx = cadd(cscale(gcx, hr), cmul(cconj(gcx), x2h));
        const float2 gxy = cadd(cscale(gcy, hr), cmul(cconj(gcy), x2h));
        dj = fmaf(gcx.x, xh.x, fmaf(gcx.y, xh.y, dj));
        dj1 = fmaf(gcy.x, xh.x, fmaf(gcy.y, xh.y, dj1));
        gfa = cscale(cmul(cconj(gxx), fb), sca);  // real channel: d(dx)
        gfb = cscale(cmul(cconj(gxy), fb), sca);  // imaginary channel: d(dy)
      }
      v[e] = make_float2(gfa.x - gfb.y, gfa.y + gfb.x);  // Q(ky, w) = G_FA + i G_FB
      // the mirrored column's bin N - ky, Q(N - ky, N - w) = conj(G_FA(ky, w))
      // + i conj(G_FB(ky, w)), goes to slot A (free; slot B still holds mirror
      // spectra other lanes read), so no gradient is held in registers
      slotA[lidx((N - ky) & (N - 1))] = make_float2(gfa.x + gfb.y, gfb.x - gfa.y);
    }
    wave_lds_sync();
    // twiddles loaded only now: they are not live during the gradient loop
    Twiddles<N> tw;
    tw_load<N>(tw, t, a.tw);
    float2* dst = a.Y + (size_t)pair * N * N;
    fft_wave<N, true>(v, slotB, t, tw);  // slot B is free once the loop is done
#pragma unroll
    for (int e = 0; e < E; ++e) dst[(size_t)w * N + t + e * T] = v[e];
    if (wm != w) {
#pragma unroll
      for (int e = 0; e < E; ++e) u[e] = slotA[lidx(t + e * T)];
      wave_lds_sync();
      fft_wave<N, true>(u, slotA, t, tw);
#pragma unroll
      for (int e = 0; e < E; ++e) dst[(size_t)wm * N + t + e * T] = u[e];
    }
  }
  // per-workgroup partials of dJ/d(eps^2) and of the Hessian sums
  const float vals[kDpart] = {wave_sum_f32(dj), wave_sum_f32(dj1), wave_sum_f32(hxx), wave_sum_f32(hyy),
                              wave_sum_f32(hxy), 0.0f};
  if ((tid & 63) == 0) {
#pragma unroll
    for (int q = 0; q < kDpart; ++q) red[tid >> 6][q] = (double)vals[q];
  }
  __syncthreads();
  if (tid < kDpart)
    a.dpart[((size_t)pair * NW + wg) * kDpart + tid] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
}

// ---------------------------------------------------------------- row stage
// Per image, the 20 pixel sums of the header comment; acc layout:
// [0..5] P1, [6..11] P2, [12..17] P3, [18] Q, [19] R.  In CJ mode the second
// channel differentiates the same image A, so it shares P2, P3 and R with the
// first and keeps only its own P1 and Q (layout [0..5] P1, [18] Q).
//
// The block's R window rows: the inverse row FFTs of G_w first (both
// channels, written back to the stage), then one pass over the pixels per
// image, sampled as in the forward row pass (uint8 source tile in LDS when
// the footprint fits, per-row FP64 parameters with FP32 per-pixel offsets,
// constant weights for translation windows).
// Per-pixel offsets of the sample point from the row's point at u = 0: u a
// split into u round(a), an exact integer, and u (a - round(a)), small enough
// that FP32 keeps it to ~1e-7 px.  The derivative of the bilinear sample jumps
// at integer coordinates, so the cell must be chosen as FP64 would.
template <int XV>
struct PixelOffsets {
  int ix[XV], iy[XV];
  float fx[XV], fy[XV];
};

template <int N, int R, bool TILE, bool TRANS, bool TWO, bool TO>
__device__ __forceinline__ void bwd_pixels(const float2* __restrict__ stage, int RS, const uint32_t* __restrict__ tile,
                                           const TileGeom& g, const RowParam* __restrict__ rp,
                                           const float* __restrict__ trow, const PixelOffsets<GatherCfg<N>::XV>& ku,
                                           const float (&tx)[GatherCfg<N>::XV], const swift_image& im, int y0,
                                           int tid, float off, float mean_off, bool ch1, float (&acc)[kBwdSums],
                                           float (&acc2)[kBwdSums]) {
  constexpr int XV = GatherCfg<N>::XV, RPI = GatherCfg<N>::RPI, ITER = R / RPI;
  const int rowb = g.wt4 * 4;
  const gptr<unsigned char> base = to_global<unsigned char>(im.data);
  const int xt = tid % N, r0 = (RPI > 1 ? tid / N : 0) * ITER;
#pragma unroll
  for (int c = 0; c < XV; ++c) {
    const int x = xt + 256 * c;
    const float u = (float)(x - N / 2);
    uint32_t prev = 0;  // translation windows: the tile byte pair of the previous row's bottom
    // the column's sums without the factor u (u is the same down the column):
    // tg ax, tg ay, tap ax, tap ay, tw ax, tw ay, and tg2 ax, tg2 ay
    float cs[6] = {0, 0, 0, 0, 0, 0}, cs2[2] = {0, 0};
#pragma unroll 2
    for (int i = 0; i < ITER; ++i) {
      const int r = r0 + i;
      const RowParam p = rp[TRANS ? r0 : r];
      float fx, fy, i00, i10, i01, i11;
      if constexpr (TRANS) {
        // same weights for every pixel; rows step by one tile row
        fx = p.fx;
        fy = p.fy;
        const int ix = min(max(p.bx + (x - N / 2), 0), rowb - 2);
        const int iy = p.by + i;
        const uint32_t vt = i == 0 ? tile_pair(tile, min(max(iy, 0), g.ht - 1) * rowb + ix) : prev;
        const uint32_t vb = tile_pair(tile, min(max(iy + 1, 0), g.ht - 1) * rowb + ix);
        prev = vb;
        i00 = (float)(vt & 255u);
        i10 = (float)((vt >> 8) & 255u);
        i01 = (float)(vb & 255u);
        i11 = (float)((vb >> 8) & 255u);
      } else {
        const float xr = p.fx + ku.fx[c], yr = p.fy + ku.fy[c];
        const float xf = floorf(xr), yf = floorf(yr);
        fx = xr - xf;
        fy = yr - yf;
        const int x0 = p.bx + ku.ix[c] + (int)xf, yy0 = p.by + ku.iy[c] + (int)yf;
        if constexpr (TILE) {
          const int ix = min(max(x0, 0), rowb - 2), iy = min(max(yy0, 0), g.ht - 2);
          const int off = iy * rowb + ix;
          const uint32_t vt = tile_pair(tile, off), vb = tile_pair(tile, off + rowb);
          i00 = (float)(vt & 255u);
          i10 = (float)((vt >> 8) & 255u);
          i01 = (float)(vb & 255u);
          i11 = (float)((vb >> 8) & 255u);
        } else {
          const int cx0 = min(max(x0, 0), im.width - 1), cx1 = min(max(x0 + 1, 0), im.width - 1);
          const int cy0 = min(max(yy0, 0), im.height - 1), cy1 = min(max(yy0 + 1, 0), im.height - 1);
          const gptr<unsigned char> q0 = base + (int64_t)cy0 * im.pitch;
          const gptr<unsigned char> q1 = base + (int64_t)cy1 * im.pitch;
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
        }
      }
      const float top = fmaf(fx, i10 - i00, i00), bot = fmaf(fx, i11 - i01, i01);
      const float val = fmaf(fy, bot - top, top);
      // bilinear partials (floor cell; clamped reads give zero outside)
      const float ax = (1.0f - fy) * (i10 - i00) + fy * (i11 - i01);
      const float ay = (1.0f - fx) * (i01 - i00) + fx * (i11 - i10);
      // D = (ax u, ax v, ax, ay u, ay v, ay): the v entries here, the u
      // entries from the column sums after the loop
      const float v = (float)(y0 + r - N / 2);
      const float tap = tx[c] * trow[r];
      const float wv = ((val - off) - mean_off) * tap;
      const float2 gw = stage[r * RS + lidx(x)];
      const float g0 = ch1 ? gw.y : gw.x;
      const float tg = tap * g0, tw = tap * wv;
      const float wt[3] = {tg, tap, tw};
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        cs[2 * q] = fmaf(wt[q], ax, cs[2 * q]);
        cs[2 * q + 1] = fmaf(wt[q], ay, cs[2 * q + 1]);
        if constexpr (!TO) {
          const float wq = wt[q] * v;
          acc[6 * q + 1] = fmaf(wq, ax, acc[6 * q + 1]);
          acc[6 * q + 4] = fmaf(wq, ay, acc[6 * q + 4]);
        }
      }
      acc[18] += tg;
      acc[19] += tw;
      if constexpr (TWO) {
        const float tg2 = tap * gw.y;
        cs2[0] = fmaf(tg2, ax, cs2[0]);
        cs2[1] = fmaf(tg2, ay, cs2[1]);
        if constexpr (!TO) {
          const float wq = tg2 * v;
          acc2[1] = fmaf(wq, ax, acc2[1]);
          acc2[4] = fmaf(wq, ay, acc2[4]);
        }
        acc2[18] += tg2;
      }
    }
    // translation-only: the u and v entries stay zero
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      acc[6 * q + 2] += cs[2 * q];
      acc[6 * q + 5] += cs[2 * q + 1];
      if constexpr (!TO) {
        acc[6 * q + 0] = fmaf(u, cs[2 * q], acc[6 * q + 0]);
        acc[6 * q + 3] = fmaf(u, cs[2 * q + 1], acc[6 * q + 3]);
      }
    }
    if constexpr (TWO) {
      acc2[2] += cs2[0];
      acc2[5] += cs2[1];
      if constexpr (!TO) {
        acc2[0] = fmaf(u, cs2[0], acc2[0]);
        acc2[3] = fmaf(u, cs2[1], acc2[3]);
      }
    }
  }
}

template <int N, bool TWO, bool TO>
__device__ __forceinline__ void bwd_image(const float2* stage, int RS, uint32_t* tile, const TileGeom& g,
                                          const RowParam* rp, const float* trow,
                                          const PixelOffsets<GatherCfg<N>::XV>& ku,
                                          const float (&tx)[GatherCfg<N>::XV], const swift_image& im, bool trans,
                                          int y0, int tid, float off, float mean_off, bool ch1,
                                          float (&acc)[kBwdSums], float (&acc2)[kBwdSums]) {
  constexpr int R = BwdRowsCfg<N>::R;
  if (g.use) {
    if (trans)
      bwd_pixels<N, R, true, true, TWO, TO>(stage, RS, tile, g, rp, trow, ku, tx, im, y0, tid, off, mean_off, ch1, acc, acc2);
    else
      bwd_pixels<N, R, true, false, TWO, TO>(stage, RS, tile, g, rp, trow, ku, tx, im, y0, tid, off, mean_off, ch1,
                                         acc, acc2);
  } else {
    bwd_pixels<N, R, false, false, TWO, TO>(stage, RS, tile, g, rp, trow, ku, tx, im, y0, tid, off, mean_off, ch1, acc, acc2);
  }
}

template <int N, bool CJ, bool TO>
__global__ void __launch_bounds__(256) k_bwd_row(BwdArgs a) {
  using C = FftCfg<N>;
  constexpr int T = C::T, E = C::E, G = 256 / T, R = BwdRowsCfg<N>::R, NSLICE = N / R;
  constexpr int RS = rows_stride<R>(fft_scratch<N>());
  constexpr int BUDGET = BwdRowsCfg<N>::TILE, XV = GatherCfg<N>::XV;
  static_assert(R % G == 0 && 2 * R <= 64, "row split");
  __shared__ float2 stage[R * RS];
  __shared__ __align__(16) uint32_t tile[BUDGET > 0 ? BUDGET / 4 + 1 : 1];  // + 1: tile_pair reads the dword after a pair
  __shared__ RowParam rparam[2][R];
  __shared__ float trow[R];
  __shared__ double red[4][2 * kBwdSums];

  const int blk = xcd_block(blockIdx.x, gridDim.x);
  const int pair = blk / NSLICE, slice = blk % NSLICE, y0 = slice * R;
  const int tid = threadIdx.x, gi = tid / T, t = tid % T;

  // sampling set-up of both images (as in the forward row pass)
  const int ka = min(max(a.img_a[pair], 0), a.n_imgs - 1);
  const int kb = min(max(a.img_b[pair], 0), a.n_imgs - 1);
  swift_image im[2] = {a.imgs[ka], a.imgs[kb]};
  const float* th[2] = {a.th_a + 8 * (size_t)pair, a.th_b + 8 * (size_t)pair};
  RowAffine ra[2];
  TileGeom tg[2];
  bool border[2];
#pragma unroll
  for (int m = 0; m < 2; ++m) {
    im[m].width = max(im[m].width, 2);
    im[m].height = max(im[m].height, 2);
    ra[m] = row_affine(th[m]);
    tg[m] = tile_geom<N, R, BUDGET, BwdRowsCfg<N>::TRW>(ra[m], im[m], y0);
    // tiles that reach past the image edge need their edge bytes replicated
    border[m] = !(tg[m].use && tg[m].xlo >= 0 && tg[m].xlo + 4 * tg[m].wt4 <= im[m].width &&
                  tg[m].ylo >= 0 && tg[m].ylo + tg[m].ht <= im[m].height);
  }
  constexpr int TRW = BwdRowsCfg<N>::TRW;
  uint4 bufA[TRW], bufB[TRW];
  if (tg[0].use) tile_fetch<tile_cw<N>()>(bufA, tg[0], im[0], tid);
  if (!CJ && tg[1].use) tile_fetch<tile_cw<N>()>(bufB, tg[1], im[1], tid);
  if (tid < 2 * R) {
    const bool mb = tid >= R;
    const int r = tid % R;
    const double xc = mb ? ra[1].xc : ra[0].xc, yc = mb ? ra[1].yc : ra[0].yc;
    const double a12 = mb ? ra[1].a12 : ra[0].a12, a22 = mb ? ra[1].a22 : ra[0].a22;
    const int xo = mb ? (tg[1].use ? tg[1].xlo : 0) : (tg[0].use ? tg[0].xlo : 0);
    const int yo = mb ? (tg[1].use ? tg[1].ylo : 0) : (tg[0].use ? tg[0].ylo : 0);
    const double v = (double)(y0 + r - N / 2);
    const double X = fmin(fmax(xc + a12 * v, -1e9), 1e9);
    const double Y = fmin(fmax(yc + a22 * v, -1e9), 1e9);
    const double bxd = floor(X), byd = floor(Y);
    RowParam p;
    p.bx = (int)bxd - xo;
    p.by = (int)byd - yo;
    p.fx = (float)(X - bxd);
    p.fy = (float)(Y - byd);
    rparam[mb ? 1 : 0][r] = p;
  } else if (tid >= 64 && tid < 64 + R) {
    trow[tid - 64] = a.taper[y0 + tid - 64];
  }
  float tx[XV];
  PixelOffsets<XV> ku[2];
#pragma unroll
  for (int c = 0; c < XV; ++c) {
    const int x = tid % N + 256 * c;
    const float u = (float)(x - N / 2);
    tx[c] = a.taper[x];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const float rx = rintf(ra[m].f11), ry = rintf(ra[m].f21);
      ku[m].ix[c] = (int)(rx * u);
      ku[m].iy[c] = (int)(ry * u);
      ku[m].fx[c] = (ra[m].f11 - rx) * u;
      ku[m].fy[c] = (ra[m].f21 - ry) * u;
    }
  }
  const bool trans[2] = {ra[0].a11 == 1.0 && ra[0].a12 == 0.0 && ra[0].a21 == 0.0 && ra[0].a22 == 1.0,
                         ra[1].a11 == 1.0 && ra[1].a12 == 0.0 && ra[1].a21 == 0.0 && ra[1].a22 == 1.0};

  // stage[r][kx] = Y[kx][y0 + r], then the inverse row FFTs of G_w in place
  const float2* Yp = a.Y + (size_t)pair * N * N;
  if constexpr (256 % (32 * R) == 0) {
    // thread: row r = tid % R of columns c0 + k CPL (CPL a multiple of 32, so
    // the stage index advances by the constant lidx(CPL)); the global address
    // is the pair's base plus a 32-bit offset
    constexpr int CPL = 256 / R, LD = N / CPL;
    const int r = tid % R, c0 = tid / R;
    const char* yb = reinterpret_cast<const char*>(Yp);
    const uint32_t off0 = (uint32_t)(c0 * N + y0 + r) * (uint32_t)sizeof(float2);
    float2 buf[LD];
#pragma unroll
    for (int k = 0; k < LD; ++k)
      buf[k] = *reinterpret_cast<const float2*>(yb + off0 + (uint32_t)(k * CPL * N * sizeof(float2)));
    float2* sp = stage + r * RS + lidx(c0);
#pragma unroll
    for (int k = 0; k < LD; ++k) sp[k * lidx(CPL)] = buf[k];
  } else {
    constexpr int LD = (N * R + 255) / 256;
    float2 buf[LD];
#pragma unroll
    for (int k = 0; k < LD; ++k) {
      const int idx = min(tid + 256 * k, N * R - 1);
      buf[k] = Yp[(size_t)(idx / R) * N + y0 + idx % R];
    }
#pragma unroll
    for (int k = 0; k < LD; ++k) {
      const int idx = tid + 256 * k;
      if (idx < N * R) stage[(idx % R) * RS + lidx(idx / R)] = buf[k];
    }
  }
  __syncthreads();
  {
    Twiddles<N> tw;
    tw_load<N>(tw, t, a.tw);
#pragma unroll 1
    for (int it = 0; it < R / G; ++it) {
      float2* row = stage + (gi + it * G) * RS;
      float2 v[E];
#pragma unroll
      for (int e = 0; e < E; ++e) v[e] = row[lidx(t + e * T)];
      wave_lds_sync();
      fft_wave<N, true>(v, row, t, tw);  // real / imaginary channel at x = t + e T
      wave_lds_sync();
#pragma unroll
      for (int e = 0; e < E; ++e) row[lidx(t + e * T)] = v[e];
    }
  }

  const PairStat ps = a.ps[pair];
  float acc0[kBwdSums], acc1[kBwdSums];
#pragma unroll
  for (int j = 0; j < kBwdSums; ++j) acc0[j] = acc1[j] = 0.0f;
  if (tg[0].use) tile_store<tile_cw<N>()>(tile, bufA, tg[0], im[0], border[0], tid);
  __syncthreads();  // G rows and tile A visible
  // image A: channel 0 (and, in CJ mode, channel 1 on the same pixels)
  // w = ((a - o) - m) T: o the offset, m the weighted mean of a - o
  bwd_image<N, CJ, TO>(stage, RS, tile, tg[0], rparam[0], trow, ku[0], tx, im[0], trans[0], y0, tid, ps.oA, ps.mA,
                       false, acc0, acc1);
  if constexpr (!CJ) {
    __syncthreads();  // tile A consumed
    if (tg[1].use) tile_store<tile_cw<N>()>(tile, bufB, tg[1], im[1], border[1], tid);
    __syncthreads();
    bwd_image<N, false, false>(stage, RS, tile, tg[1], rparam[1], trow, ku[1], tx, im[1], trans[1], y0, tid,
                               ps.oB, ps.mB, true, acc1, acc1);
  }
  // block reduction to FP64 slice partials
  const int wv = tid >> 6, ln = tid & 63;
#pragma unroll
  for (int j = 0; j < kBwdSums; ++j) {
    // translation only: the tx / ty entries of P1, P2, P3 (j % 6 = 2, 5), Q
    // and R; the others are zero and are not reduced
    const bool used = !TO || j >= 18 || j % 6 == 2 || j % 6 == 5;
    const float sa = used ? wave_sum_f32(acc0[j]) : 0.0f;
    // CJ: channel 1 shares P2, P3 and R with channel 0
    const bool own = !CJ || j < 6 || j == 18;
    const float sb = own ? (used ? wave_sum_f32(acc1[j]) : 0.0f) : sa;
    if (ln == 0) {
      red[wv][j] = (double)sa;
      red[wv][kBwdSums + j] = (double)sb;
    }
  }
  __syncthreads();
  if (tid < 2 * kBwdSums)
    a.rpart[((size_t)pair * NSLICE + slice) * 2 * kBwdSums + tid] = red[0][tid] + red[1][tid] + red[2][tid] + red[3][tid];
}

// ---------------------------------------------------------------- per pair
template <int N, bool CJ>
__global__ void __launch_bounds__(64) k_bwd_fin(BwdArgs a) {
  constexpr int NW = bwd_col_blocks<N>();
  constexpr int NSLICE = N / BwdRowsCfg<N>::R;
  __shared__ double tot[2 * kBwdSums];
  const int pair = blockIdx.x, ln = threadIdx.x;
  double dj = 0.0, dj1 = 0.0, hs[3] = {0.0, 0.0, 0.0};
  for (int i = ln; i < NW; i += 64) {
    const double* q = a.dpart + ((size_t)pair * NW + i) * kDpart;
    dj += q[0];
    dj1 += q[1];
    hs[0] += q[2];
    hs[1] += q[3];
    hs[2] += q[4];
  }
  dj = wave_sum(dj);
  dj1 = wave_sum(dj1);
  hs[0] = wave_sum(hs[0]);
  hs[1] = wave_sum(hs[1]);
  hs[2] = wave_sum(hs[2]);
  if (!CJ && a.peak_hess && ln < 3) {
    // d2c/ds2 = -(2 pi / N)^2 / M sum C(k) f f' e^{+i phi}, C = X h
    const double sc = -4.0 * M_PI * M_PI / ((double)N * N * (double)N * N);
    a.peak_hess[(size_t)pair * 3 + ln] = (float)(sc * hs[ln]);
  }
  if (ln < 2 * kBwdSums) {
    double s = 0.0;
    for (int sl = 0; sl < NSLICE; ++sl) s += a.rpart[((size_t)pair * NSLICE + sl) * 2 * kBwdSums + ln];
    tot[ln] = s;
  }
  __syncthreads();
  if (ln < 12) {
    const int img = ln / 6, j = ln % 6;
    const PairStat ps = a.ps[pair];
    const TaperInfo ti = *a.tinfo;
    const double sT = ti.sum_t * ti.sum_t;
    const double e2 = (double)a.eps_rel * (double)a.eps_rel;
    // eps^2 = eps_rel^2 |w_A|^2 |w_B|^2: each channel's lambda multiplies the
    // differentiated window's w by the other window's norm; dJ/d(eps^2) is
    // s^(p+1) times the column stage's normalised sums, s = 1 / (|w_A| |w_B|)
    const double sp1 = (ps.flags & 1) ? 0.0 : pow((double)ps.swA * (double)ps.swB, -0.5 * ((double)a.p + 1.0));
    const double lam = CJ ? (img == 0 ? dj : dj1) * sp1 * 2.0 * e2 * (double)ps.swB
                          : dj * sp1 * 2.0 * e2 * (img == 0 ? (double)ps.swB : (double)ps.swA);
    const double* q = tot + img * kBwdSums;
    double g = q[j] + lam * q[12 + j] - (q[18] + lam * q[19]) / sT * q[6 + j];
    if (ps.flags & 1) g = 0.0;
    if (CJ) {
      a.jac[((size_t)pair * 2 + img) * 6 + j] = (float)g;
    } else {
      float* dst = img == 0 ? a.g_th_a : a.g_th_b;
      if (dst) dst[(size_t)pair * 6 + j] = (float)g;
    }
  }
}

// ---------------------------------------------------------------- launcher
template <int N, bool CJ>
static hipError_t launch_bwd_t(const BwdArgs& a, hipStream_t s, KernelTimer* kt) {
  constexpr int NW = bwd_col_blocks<N>();
  constexpr int NSLICE = N / BwdRowsCfg<N>::R;
  const unsigned P = (unsigned)a.npairs;
  if (kt) kt->begin(CJ ? "k_cj_col" : "k_bwd_col", N, s);
  k_bwd_col<N, CJ><<<P * NW, 256, 0, s>>>(a);
  if (kt) kt->end(s);
  if (kt) kt->begin(CJ ? "k_cj_row" : "k_bwd_row", N, s);
  if constexpr (CJ) {
    if (a.jac_trans)
      k_bwd_row<N, true, true><<<P * NSLICE, 256, 0, s>>>(a);
    else
      k_bwd_row<N, true, false><<<P * NSLICE, 256, 0, s>>>(a);
  } else {
    k_bwd_row<N, false, false><<<P * NSLICE, 256, 0, s>>>(a);
  }
  if (kt) kt->end(s);
  if (kt) kt->begin(CJ ? "k_cj_fin" : "k_bwd_fin", N, s);
  k_bwd_fin<N, CJ><<<P, 64, 0, s>>>(a);
  if (kt) kt->end(s);
  return hipGetLastError();
}

template <bool CJ>
static hipError_t launch_bwd_n(int n, const BwdArgs& a, hipStream_t s, KernelTimer* kt) {
  switch (n) {
    case 64: return launch_bwd_t<64, CJ>(a, s, kt);
    case 128: return launch_bwd_t<128, CJ>(a, s, kt);
    case 256: return launch_bwd_t<256, CJ>(a, s, kt);
    case 512: return launch_bwd_t<512, CJ>(a, s, kt);
    case 1024: return launch_bwd_t<1024, CJ>(a, s, kt);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_backward_group(int n, const BwdArgs& a, bool centroid_jac, hipStream_t s, KernelTimer* kt) {
  return centroid_jac ? launch_bwd_n<true>(n, a, s, kt) : launch_bwd_n<false>(n, a, s, kt);
}

int bwd_col_blocks_n(int n) {
  switch (n) {
    case 64: return bwd_col_blocks<64>();
    case 128: return bwd_col_blocks<128>();
    case 256: return bwd_col_blocks<256>();
    case 512: return bwd_col_blocks<512>();
    default: return bwd_col_blocks<1024>();
  }
}

int bwd_row_blocks_n(int n) {
  switch (n) {
    case 64: return 64 / BwdRowsCfg<64>::R;
    case 128: return 128 / BwdRowsCfg<128>::R;
    case 256: return 256 / BwdRowsCfg<256>::R;
    case 512: return 512 / BwdRowsCfg<512>::R;
    default: return 1024 / BwdRowsCfg<1024>::R;
  }
}

}  // namespace swift
