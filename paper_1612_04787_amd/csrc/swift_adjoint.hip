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

namespace swift {

// ---------------------------------------------------------------- column stage
template <int N, bool CJ>
__global__ void __launch_bounds__(256) k_bwd_col(BwdArgs a) {
  using C = FftCfg<N>;
  constexpr int T = C::T, E = C::E, G = 256 / T, IPW = G / 2;
  constexpr int NI = N / 2 + 1, NW = (NI + IPW - 1) / IPW;
  constexpr int SL = lidx(N);
  __shared__ float2 lds[G * SL];
  __shared__ double red[4][kDpart];

  const int pair = blockIdx.x / NW, wg = blockIdx.x % NW;
  const int tid = threadIdx.x, c = tid / T, t = tid % T;
  const int which = c / IPW, item = c % IPW, w = wg * IPW + item;
  const bool valid = w < NI;
  const int col = which == 0 ? w : ((N - w) & (N - 1));
  float2* slotA = lds + item * SL;          // transform of column w
  float2* slotB = lds + (item + IPW) * SL;  // transform of column N - w
  float2 v[E];
  Twiddles<N> tw;
  tw_load<N>(tw, t, a.tw);
  float2 tau[E];
  if (valid) {
    const float2* src = a.Zf + (size_t)pair * N * N + (size_t)col * N;
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = src[t + e * T];
#pragma unroll
    for (int e = 0; e < E; ++e) tau[e] = a.tau[t + e * T];
    if (which == 1) {
#pragma unroll
      for (int e = 0; e < E; ++e) slotB[lidx(t + e * T)] = v[e];
    }
  }
  __syncthreads();

  float dj = 0.0f, dj1 = 0.0f, hxx = 0.0f, hyy = 0.0f, hxy = 0.0f;
  float2 gb[E];
  if (valid && which == 0) {
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
    }
    const float p = a.p, hp2 = -0.5f * p;
    const float inv_m = 1.0f / (float)(N * N);
    const float mw = (w == 0 || w == N / 2) ? 1.0f : 2.0f;  // column w and its mirror N - w
    const float2 tauw = a.tau[w];
    // signed frequency of the column (Nyquist: squared terms only)
    const float fw = (float)w, fwm = (w == N / 2) ? 0.0f : (float)w;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int ky = t + e * T;
      const float2 zp = v[e];
      const float2 zm = cconj(slotB[lidx((N - ky) & (N - 1))]);
      float2 fa = cscale(cadd(zp, zm), 0.5f);
      const float2 dd = csub(zp, zm);
      float2 fb = make_float2(0.5f * dd.y, -0.5f * dd.x);
      const float2 tk = cmul(tau[e], tauw);
      fa = csub(fa, cscale(tk, ps.mA));
      fb = csub(fb, cscale(tk, ps.mB));
      const float2 X = make_float2(fa.x * fb.x + fa.y * fb.y, fa.x * fb.y - fa.y * fb.x);
      const float r = X.x * X.x + X.y * X.y;
      const float d = r + ps.eps2;
      float h, hd;  // h and h' = dh/dd
      if (p == 0.0f) {
        h = 1.0f;
        hd = 0.0f;
      } else if (!(d > 0.0f)) {
        h = 0.0f;
        hd = 0.0f;
      } else {
        h = (p == 1.0f) ? __builtin_amdgcn_rsqf(d) : __builtin_amdgcn_exp2f(hp2 * __builtin_amdgcn_logf(d));
        hd = hp2 * h / d;
      }
      // e^{-2 pi i (ky iy + w ix) / N} from the W_1024 table
      const int m = (ky * rec.iy + w * rec.ix) & (N - 1);
      const float2 ph = a.tw[m * (1024 / N)];
      // surface Hessian sums: Re(X h e^{+i phi}) times the frequency products
      if (!zero_all && !(ky == 0 && w == 0)) {
        const float2 cc = cmul(cscale(X, h), cconj(ph));
        const float fy = (ky < N / 2) ? (float)ky : (float)(ky - N);
        const float fym = (ky == N / 2) ? 0.0f : fy;
        hxx += mw * cc.x * fw * fw;
        hyy += mw * cc.x * fy * fy;
        hxy += mw * cc.x * fwm * fym;
      }
      const float2 x2 = cmul(X, X);
      const bool zb = zero_all || (ky == 0 && w == 0);
      float2 gfa, gfb;
      if constexpr (!CJ) {
        float2 gc = cscale(cadd(cscale(ph, alpha), cscale(X, gamma * h)), inv_m);
        if (zb) gc = make_float2(0.0f, 0.0f);
        // G_X = G_C (h + r h') + conj(G_C) X^2 h'
        const float2 gx = cadd(cscale(gc, h + r * hd), cscale(cmul(cconj(gc), x2), hd));
        dj += mw * cmul(cconj(gc), X).x * hd;
        gfa = cmul(cconj(gx), fb);
        gfb = cmul(gx, fa);
      } else {
        // 3 x 3 sums S = sum omega e_x^dx e_y^dy with e = e^{-2 pi i k/N}
        const float2 ex = a.tw[w * (1024 / N)], ey = a.tw[ky * (1024 / N)];
        const float2 exc = cconj(ex), eyc = cconj(ey);
        float2 sx = make_float2(0.f, 0.f), sy = make_float2(0.f, 0.f);
#pragma unroll
        for (int r3 = 0; r3 < 3; ++r3) {
          const float2 rx = cadd(cadd(cscale(exc, omx[3 * r3]), make_float2(omx[3 * r3 + 1], 0.f)),
                                 cscale(ex, omx[3 * r3 + 2]));
          const float2 ry = cadd(cadd(cscale(exc, omy[3 * r3]), make_float2(omy[3 * r3 + 1], 0.f)),
                                 cscale(ex, omy[3 * r3 + 2]));
          const float2 ef = r3 == 0 ? eyc : (r3 == 1 ? make_float2(1.f, 0.f) : ey);
          sx = cadd(sx, cmul(rx, ef));
          sy = cadd(sy, cmul(ry, ef));
        }
        float2 gcx = cscale(cmul(ph, sx), inv_m), gcy = cscale(cmul(ph, sy), inv_m);
        if (zb) gcx = gcy = make_float2(0.0f, 0.0f);
        const float2 gxx = cadd(cscale(gcx, h + r * hd), cscale(cmul(cconj(gcx), x2), hd));
        const float2 gxy = cadd(cscale(gcy, h + r * hd), cscale(cmul(cconj(gcy), x2), hd));
        dj += mw * cmul(cconj(gcx), X).x * hd;
        dj1 += mw * cmul(cconj(gcy), X).x * hd;
        gfa = cmul(cconj(gxx), fb);  // real channel: d(dx)
        gfb = cmul(cconj(gxy), fb);  // imaginary channel: d(dy)
      }
      v[e] = make_float2(gfa.x - gfb.y, gfa.y + gfb.x);  // Q(ky, w) = G_FA + i G_FB
      // keep G_FA, G_FB of column w for the mirrored column (read after the barrier)
      tau[e] = gfa;
      gb[e] = gfb;
    }
    // slot B is overwritten only after every lane of this wave has read its mirror value
    wave_lds_sync();
#pragma unroll
    for (int e = 0; e < E; ++e) {
      slotA[lidx(t + e * T)] = tau[e];
      slotB[lidx(t + e * T)] = gb[e];
    }
  }
  __syncthreads();
  if (valid && which == 1) {
    // Q(ky, N - w) = conj(G_FA(-ky, w)) + i conj(G_FB(-ky, w))
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int ky = t + e * T;
      const float2 ga = cconj(slotA[lidx((N - ky) & (N - 1))]);
      const float2 gb = cconj(slotB[lidx((N - ky) & (N - 1))]);
      v[e] = make_float2(ga.x - gb.y, ga.y + gb.x);
    }
  }
  __syncthreads();
  if (valid && (which == 0 || col != w)) {
    fft_wave<N, true>(v, which == 0 ? slotA : slotB, t, tw);
    float2* dst = a.Y + (size_t)pair * N * N + (size_t)col * N;
#pragma unroll
    for (int e = 0; e < E; ++e) dst[t + e * T] = v[e];
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
// [0..5] P1, [6..11] P2, [12..17] P3, [18] Q, [19] R.
struct PixelTerms {
  float D[6];  // (a_x u, a_x v, a_x, a_y u, a_y v, a_y)
  float tap;   // T
  float w;     // (a - m) T
};

template <int N>
__device__ __forceinline__ PixelTerms bwd_terms(const swift_image& im, const float* th, double vrow, int x,
                                                float tap, float mean_off, bool& cl) {
  const double u = (double)(x - N / 2);
  const double X = fmin(fmax((double)th[0] + (double)th[4] + (double)th[2] * u + (double)th[3] * vrow, -1e9), 1e9);
  const double Y = fmin(fmax((double)th[1] + (double)th[7] + (double)th[5] * u + (double)th[6] * vrow, -1e9), 1e9);
  const double xfd = floor(X), yfd = floor(Y);
  const float fx = (float)(X - xfd), fy = (float)(Y - yfd);
  const int x0 = (int)xfd, y0 = (int)yfd;
  cl |= (x0 < 0) | (x0 > im.width - 2) | (y0 < 0) | (y0 > im.height - 2);
  const int cx0 = min(max(x0, 0), im.width - 1), cx1 = min(max(x0 + 1, 0), im.width - 1);
  const int cy0 = min(max(y0, 0), im.height - 1), cy1 = min(max(y0 + 1, 0), im.height - 1);
  const gptr<unsigned char> base = to_global<unsigned char>(im.data);
  const gptr<unsigned char> r0 = base + (int64_t)cy0 * im.pitch;
  const gptr<unsigned char> r1 = base + (int64_t)cy1 * im.pitch;
  float i00, i10, i01, i11;
  if (im.dtype == SWIFT_U8) {
    i00 = (float)r0[cx0];
    i10 = (float)r0[cx1];
    i01 = (float)r1[cx0];
    i11 = (float)r1[cx1];
  } else {
    i00 = ((gptr<float>)r0)[cx0];
    i10 = ((gptr<float>)r0)[cx1];
    i01 = ((gptr<float>)r1)[cx0];
    i11 = ((gptr<float>)r1)[cx1];
  }
  const float top = fmaf(fx, i10 - i00, i00), bot = fmaf(fx, i11 - i01, i01);
  const float val = fmaf(fy, bot - top, top);
  // bilinear partials (floor cell; clamped reads give zero outside)
  const float ax = (1.0f - fy) * (i10 - i00) + fy * (i11 - i01);
  const float ay = (1.0f - fx) * (i01 - i00) + fx * (i11 - i10);
  PixelTerms p;
  const float uf = (float)u, vf = (float)vrow;
  p.D[0] = ax * uf;
  p.D[1] = ax * vf;
  p.D[2] = ax;
  p.D[3] = ay * uf;
  p.D[4] = ay * vf;
  p.D[5] = ay;
  p.tap = tap;
  p.w = (val - kSampleOffset - mean_off) * tap;
  return p;
}

__device__ __forceinline__ void bwd_accumulate(float (&acc)[kBwdSums], const PixelTerms& p, float gw) {
  const float tg = p.tap * gw, tw = p.tap * p.w;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    acc[j] = fmaf(tg, p.D[j], acc[j]);
    acc[6 + j] = fmaf(p.tap, p.D[j], acc[6 + j]);
    acc[12 + j] = fmaf(tw, p.D[j], acc[12 + j]);
  }
  acc[18] += tg;
  acc[19] += tw;
}

template <int N, bool CJ>
__global__ void __launch_bounds__(256) k_bwd_row(BwdArgs a) {
  using C = FftCfg<N>;
  constexpr int T = C::T, E = C::E, G = 256 / T, R = RowsCfg<N>::FWD, NSLICE = N / R;
  constexpr int RS = lidx(N) + 1;
  static_assert(R % G == 0, "row split");
  __shared__ float2 stage[R * RS];
  __shared__ double red[4][2 * kBwdSums];

  const int pair = blockIdx.x / NSLICE, slice = blockIdx.x % NSLICE, y0 = slice * R;
  const int tid = threadIdx.x, gi = tid / T, t = tid % T;
  const float2* Yp = a.Y + (size_t)pair * N * N;
  // stage[r][kx] = Y[kx][y0 + r]
  {
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

  const int ka = min(max(a.img_a[pair], 0), a.n_imgs - 1);
  const int kb = min(max(a.img_b[pair], 0), a.n_imgs - 1);
  swift_image imA = a.imgs[ka], imB = a.imgs[kb];
  imA.width = max(imA.width, 2);
  imA.height = max(imA.height, 2);
  imB.width = max(imB.width, 2);
  imB.height = max(imB.height, 2);
  const float* thA = a.th_a + 8 * (size_t)pair;
  const float* thB = a.th_b + 8 * (size_t)pair;
  const PairStat ps = a.ps[pair];
  float acc0[kBwdSums], acc1[kBwdSums];
#pragma unroll
  for (int j = 0; j < kBwdSums; ++j) acc0[j] = acc1[j] = 0.0f;
  bool cl = false;
  Twiddles<N> tw;
  tw_load<N>(tw, t, a.tw);

#pragma unroll 1
  for (int it = 0; it < R / G; ++it) {
    const int r = gi + it * G, y = y0 + r;
    float2* row = stage + r * RS;
    float2 v[E];
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = row[lidx(t + e * T)];
    wave_lds_sync();
    fft_wave<N, true>(v, row, t, tw);  // real / imaginary channel at x = t + e T
    // park the transformed row in LDS (each lane its own elements) so that the
    // pixel loop below indexes LDS, not a register array
    wave_lds_sync();
#pragma unroll
    for (int e = 0; e < E; ++e) row[lidx(t + e * T)] = v[e];
    const float ty = a.taper[y];
    const double vrow = (double)(y - N / 2);
#pragma unroll 2
    for (int e = 0; e < E; ++e) {
      const int x = t + e * T;
      const float2 g = row[lidx(x)];
      const float tap = a.taper[x] * ty;
      const PixelTerms pa = bwd_terms<N>(imA, thA, vrow, x, tap, ps.mA, cl);
      bwd_accumulate(acc0, pa, g.x);
      if constexpr (CJ) {
        bwd_accumulate(acc1, pa, g.y);
      } else {
        const PixelTerms pb = bwd_terms<N>(imB, thB, vrow, x, tap, ps.mB, cl);
        bwd_accumulate(acc1, pb, g.y);
      }
    }
  }
  // block reduction to FP64 slice partials
  const int wv = tid >> 6, ln = tid & 63;
#pragma unroll
  for (int j = 0; j < kBwdSums; ++j) {
    const float sa = wave_sum_f32(acc0[j]);
    const float sb = wave_sum_f32(acc1[j]);
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
  constexpr int G = 256 / FftCfg<N>::T, IPW = G / 2, NW = (N / 2 + 1 + IPW - 1) / IPW;
  constexpr int NSLICE = N / RowsCfg<N>::FWD;
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
    // differentiated window's w by the other window's norm
    const double lam = CJ ? (img == 0 ? dj : dj1) * 2.0 * e2 * (double)ps.swB
                          : dj * 2.0 * e2 * (img == 0 ? (double)ps.swB : (double)ps.swA);
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
  constexpr int G = 256 / FftCfg<N>::T, IPW = G / 2, NW = (N / 2 + 1 + IPW - 1) / IPW;
  constexpr int NSLICE = N / RowsCfg<N>::FWD;
  const unsigned P = (unsigned)a.npairs;
  if (kt) kt->begin(CJ ? "k_cj_col" : "k_bwd_col", N, s);
  k_bwd_col<N, CJ><<<P * NW, 256, 0, s>>>(a);
  if (kt) kt->end(s);
  if (kt) kt->begin(CJ ? "k_cj_row" : "k_bwd_row", N, s);
  k_bwd_row<N, CJ><<<P * NSLICE, 256, 0, s>>>(a);
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

}  // namespace swift
