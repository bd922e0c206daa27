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
#include "swift_dev.hpp"

namespace swift {

// ---------------------------------------------------------------- column stage
template <int N>
__global__ void __launch_bounds__(256) k_bwd_col(BwdArgs a) {
  using C = FftCfg<N>;
  constexpr int T = C::T, E = C::E, G = 256 / T, IPW = G / 2;
  constexpr int NI = N / 2 + 1, NW = (NI + IPW - 1) / IPW;
  constexpr int SL = lidx(N);
  __shared__ float2 lds[G * SL];
  __shared__ double red[4];

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

  float dj = 0.0f;
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
    const bool zero_all = (ps.flags & 1) != 0;
    const float p = a.p, hp2 = -0.5f * p;
    const float inv_m = 1.0f / (float)(N * N);
    const float mw = (w == 0 || w == N / 2) ? 1.0f : 2.0f;  // column w and its mirror N - w
    const float2 tauw = a.tau[w];
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
      float2 gc = cscale(cadd(cscale(ph, alpha), cscale(X, gamma * h)), inv_m);
      if (zero_all || (ky == 0 && w == 0)) gc = make_float2(0.0f, 0.0f);
      // G_X = G_C (h + r h') + conj(G_C) X^2 h'
      const float2 x2 = cmul(X, X);
      const float2 gx = cadd(cscale(gc, h + r * hd), cscale(cmul(cconj(gc), x2), hd));
      const float2 cx = cmul(cconj(gc), X);
      dj += mw * cx.x * hd;
      const float2 gfa = cmul(cconj(gx), fb);
      const float2 gfb = cmul(gx, fa);
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
  // per-workgroup partial of dJ/d(eps^2)
  const float wsum = wave_sum_f32(dj);
  if ((tid & 63) == 0) red[tid >> 6] = (double)wsum;
  __syncthreads();
  if (tid == 0) a.dpart[(size_t)pair * NW + wg] = red[0] + red[1] + red[2] + red[3];
}

// ---------------------------------------------------------------- row stage
// Per image, the 20 pixel sums of the header comment; acc layout:
// [0..5] P1, [6..11] P2, [12..17] P3, [18] Q, [19] R.
template <int N>
__device__ __forceinline__ void bwd_pixel(float (&acc)[kBwdSums], const swift_image& im, const float* th, double vrow,
                                          int x, float tap, float gw, float mean_off, bool& cl) {
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
  const float wv = (val - kSampleOffset - mean_off) * tap;  // w = (a - m) T
  const float uf = (float)u, vf = (float)vrow;
  const float D[6] = {ax * uf, ax * vf, ax, ay * uf, ay * vf, ay};
  const float tg = tap * gw, tw = tap * wv;
#pragma unroll
  for (int j = 0; j < 6; ++j) {
    acc[j] = fmaf(tg, D[j], acc[j]);
    acc[6 + j] = fmaf(tap, D[j], acc[6 + j]);
    acc[12 + j] = fmaf(tw, D[j], acc[12 + j]);
  }
  acc[18] += tg;
  acc[19] += tw;
}

template <int N>
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
  swift_image im[2] = {a.imgs[ka], a.imgs[kb]};
  im[0].width = max(im[0].width, 2);
  im[0].height = max(im[0].height, 2);
  im[1].width = max(im[1].width, 2);
  im[1].height = max(im[1].height, 2);
  const float* th[2] = {a.th_a + 8 * (size_t)pair, a.th_b + 8 * (size_t)pair};
  const PairStat ps = a.ps[pair];
  float accA[kBwdSums], accB[kBwdSums];
#pragma unroll
  for (int j = 0; j < kBwdSums; ++j) accA[j] = accB[j] = 0.0f;
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
    fft_wave<N, true>(v, row, t, tw);  // v[e].x = G_wA(x), v[e].y = G_wB(x), x = t + e T
    const float ty = a.taper[y];
    const double vrow = (double)(y - N / 2);
#pragma unroll 2
    for (int e = 0; e < E; ++e) {
      const int x = t + e * T;
      const float tap = a.taper[x] * ty;
      bwd_pixel<N>(accA, im[0], th[0], vrow, x, tap, v[e].x, ps.mA, cl);
      bwd_pixel<N>(accB, im[1], th[1], vrow, x, tap, v[e].y, ps.mB, cl);
    }
  }
  // block reduction to FP64 slice partials
  const int wv = tid >> 6, ln = tid & 63;
#pragma unroll
  for (int j = 0; j < kBwdSums; ++j) {
    const float sa = wave_sum_f32(accA[j]);
    const float sb = wave_sum_f32(accB[j]);
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
template <int N>
__global__ void __launch_bounds__(64) k_bwd_fin(BwdArgs a) {
  constexpr int G = 256 / FftCfg<N>::T, IPW = G / 2, NW = (N / 2 + 1 + IPW - 1) / IPW;
  constexpr int NSLICE = N / RowsCfg<N>::FWD;
  __shared__ double tot[2 * kBwdSums];
  const int pair = blockIdx.x, ln = threadIdx.x;
  double dj = 0.0;
  for (int i = ln; i < NW; i += 64) dj += a.dpart[(size_t)pair * NW + i];
  dj = wave_sum(dj);
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
    const double lam = dj * 2.0 * e2 * (img == 0 ? (double)ps.swB : (double)ps.swA);
    const double* q = tot + img * kBwdSums;
    double g = q[j] + lam * q[12 + j] - (q[18] + lam * q[19]) / sT * q[6 + j];
    if (ps.flags & 1) g = 0.0;
    float* dst = img == 0 ? a.g_th_a : a.g_th_b;
    if (dst) dst[(size_t)pair * 6 + j] = (float)g;
  }
}

// ---------------------------------------------------------------- launcher
template <int N>
static hipError_t launch_bwd_t(const BwdArgs& a, hipStream_t s, KernelTimer* kt) {
  constexpr int G = 256 / FftCfg<N>::T, IPW = G / 2, NW = (N / 2 + 1 + IPW - 1) / IPW;
  constexpr int NSLICE = N / RowsCfg<N>::FWD;
  const unsigned P = (unsigned)a.npairs;
  if (kt) kt->begin("k_bwd_col", N, s);
  k_bwd_col<N><<<P * NW, 256, 0, s>>>(a);
  if (kt) kt->end(s);
  if (kt) kt->begin("k_bwd_row", N, s);
  k_bwd_row<N><<<P * NSLICE, 256, 0, s>>>(a);
  if (kt) kt->end(s);
  if (kt) kt->begin("k_bwd_fin", N, s);
  k_bwd_fin<N><<<P, 64, 0, s>>>(a);
  if (kt) kt->end(s);
  return hipGetLastError();
}

hipError_t launch_backward_group(int n, const BwdArgs& a, hipStream_t s, KernelTimer* kt) {
  switch (n) {
    case 64: return launch_bwd_t<64>(a, s, kt);
    case 128: return launch_bwd_t<128>(a, s, kt);
    case 256: return launch_bwd_t<256>(a, s, kt);
    case 512: return launch_bwd_t<512>(a, s, kt);
    case 1024: return launch_bwd_t<1024>(a, s, kt);
  }
  return hipErrorInvalidValue;
}

}  // namespace swift
