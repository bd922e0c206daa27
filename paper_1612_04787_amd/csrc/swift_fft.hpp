// Wave-resident complex FFTs for gfx950 (64-lane wavefronts).
//
// One length-N transform lives inside one wavefront: T = N/E lanes each hold
// E complex values in registers.  Lane t holds element t + e*T (e < E) on entry
// and output bin t + e*T on exit (natural order in both directions).  Passes
// are Stockham autosort steps of radix R (the butterfly index j = t + b*T reads
// x[j + q*N/R] and writes y[(j/Ns)*Ns*R + j%Ns + q*Ns]); between passes the
// data goes through LDS.  Because a transform never spans two wavefronts, the
// exchange only needs wave-level ordering (LDS operations of one wavefront
// complete in issue order), not a workgroup barrier.
//
//   N     E   T   radices
//   64    8   8   8 8
//   128   8   16  8 8 2
//   256   8   32  8 8 4
//   512   8   64  8 8 8
//   1024  16  64  16 16 4
#pragma once
#include <hip/hip_runtime.h>

namespace swift {

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
// multiply by -i (forward transform) or +i (inverse transform)
template <bool INV>
__device__ __forceinline__ float2 mul_mi(float2 a) {
  return INV ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// LDS index with one padding slot every 32 complex values.  LDS has 64
// banks of 4 bytes and an 8-byte access serves 32 lanes per cycle, so any 32
// consecutive indices then fall on 32 distinct bank pairs.
__host__ __device__ constexpr int lidx(int i) { return i + (i >> 5); }

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int N> struct FftCfg;
template <> struct FftCfg<64>   { static constexpr int E = 8,  T = 8,  NP = 2; static constexpr int rad(int) { return 8; } };
template <> struct FftCfg<128>  { static constexpr int E = 8,  T = 16, NP = 3; static constexpr int rad(int p) { return p < 2 ? 8 : 2; } };
template <> struct FftCfg<256>  { static constexpr int E = 8,  T = 32, NP = 3; static constexpr int rad(int p) { return p < 2 ? 8 : 4; } };
template <> struct FftCfg<512>  { static constexpr int E = 8,  T = 64, NP = 3; static constexpr int rad(int) { return 8; } };
template <> struct FftCfg<1024> { static constexpr int E = 16, T = 64, NP = 3; static constexpr int rad(int p) { return p < 2 ? 16 : 4; } };

// ---------------------------------------------------------------- butterflies
template <int R, bool INV> struct Dft;

template <bool INV> struct Dft<2, INV> {
  __device__ __forceinline__ static void run(float2* u) {
    float2 a = u[0], b = u[1];
    u[0] = cadd(a, b);
    u[1] = csub(a, b);
  }
};

template <bool INV> struct Dft<4, INV> {
  __device__ __forceinline__ static void run(float2* u) {
    float2 t0 = cadd(u[0], u[2]), t1 = csub(u[0], u[2]);
    float2 t2 = cadd(u[1], u[3]), t3 = mul_mi<INV>(csub(u[1], u[3]));
    u[0] = cadd(t0, t2);
    u[1] = cadd(t1, t3);
    u[2] = csub(t0, t2);
    u[3] = csub(t1, t3);
  }
};

template <bool INV> struct Dft<8, INV> {
  __device__ __forceinline__ static void run(float2* u) {
    constexpr float c = 0.70710678118654752440f;
    float2 e[4] = {u[0], u[2], u[4], u[6]};
    float2 o[4] = {u[1], u[3], u[5], u[7]};
    Dft<4, INV>::run(e);
    Dft<4, INV>::run(o);
    // o[m] *= W8^(+-m)
    float2 o1 = o[1], o3 = o[3];
    if (!INV) {
      o[1] = make_float2(c * (o1.x + o1.y), c * (o1.y - o1.x));
      o[3] = make_float2(c * (o3.y - o3.x), -c * (o3.x + o3.y));
    } else {
      o[1] = make_float2(c * (o1.x - o1.y), c * (o1.x + o1.y));
      o[3] = make_float2(-c * (o3.x + o3.y), c * (o3.x - o3.y));
    }
    o[2] = mul_mi<INV>(o[2]);
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      u[m] = cadd(e[m], o[m]);
      u[m + 4] = csub(e[m], o[m]);
    }
  }
};

template <bool INV> struct Dft<16, INV> {
  __device__ __forceinline__ static void run(float2* u) {
    // 16 = 4 x 4: inner DFT4 over q1 for each q2, twiddle W16^(q2 k1), outer DFT4
    constexpr float C1 = 0.92387953251128675613f;  // cos(pi/8)
    constexpr float S1 = 0.38268343236508977173f;  // sin(pi/8)
    constexpr float C2 = 0.70710678118654752440f;
    float2 b[4][4];
#pragma unroll
    for (int q2 = 0; q2 < 4; ++q2) {
      float2 t[4] = {u[q2], u[q2 + 4], u[q2 + 8], u[q2 + 12]};
      Dft<4, INV>::run(t);
#pragma unroll
      for (int k1 = 0; k1 < 4; ++k1) b[q2][k1] = t[k1];
    }
    // W16^m for m = q2*k1 in {0,1,2,3,4,6,9}; forward uses exp(-2 pi i m / 16)
    const float sg = INV ? 1.0f : -1.0f;
    const float2 w1 = make_float2(C1, sg * S1), w2 = make_float2(C2, sg * C2), w3 = make_float2(S1, sg * C1);
    const float2 w6 = make_float2(-C2, sg * C2), w9 = make_float2(-C1, -sg * S1);
    b[1][1] = cmul(b[1][1], w1);
    b[1][2] = cmul(b[1][2], w2);
    b[1][3] = cmul(b[1][3], w3);
    b[2][1] = cmul(b[2][1], w2);
    b[2][2] = mul_mi<INV>(b[2][2]);
    b[2][3] = cmul(b[2][3], w6);
    b[3][1] = cmul(b[3][1], w3);
    b[3][2] = cmul(b[3][2], w6);
    b[3][3] = cmul(b[3][3], w9);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
      float2 t[4] = {b[0][k1], b[1][k1], b[2][k1], b[3][k1]};
      Dft<4, INV>::run(t);
#pragma unroll
      for (int k2 = 0; k2 < 4; ++k2) u[k1 + 4 * k2] = t[k2];
    }
  }
};

// ---------------------------------------------------------------- twiddles
// Pass P (P >= 1) of butterfly j = t + b*T multiplies input q by
// W_{NS*R}^(q*k), k = j mod NS.  These depend only on the lane, so kernels that
// run several transforms per lane load them once into registers.
template <int N>
__host__ __device__ constexpr int tw_off(int P) {
  int o = 0;
  for (int p = 1; p < P; ++p) o += (FftCfg<N>::E / FftCfg<N>::rad(p)) * (FftCfg<N>::rad(p) - 1);
  return o;
}
template <int N>
__host__ __device__ constexpr int tw_count() { return tw_off<N>(FftCfg<N>::NP); }

template <int N>
struct Twiddles {
  float2 w[tw_count<N>()];
};

// Index m (into W_1024^m) of register twiddle i of lane t: pass P's block of
// (E/R) (R-1) values holds, for butterfly b and input q >= 1, W_{NS R}^(q k)
// with k = (t + b T) mod NS, i.e. m = q k (1024 / (NS R)).
template <int N>
__host__ __device__ constexpr int tw_index(int t, int i) {
  using C = FftCfg<N>;
  int ns = C::rad(0);
  for (int p = 1; p < C::NP; ++p) {
    const int r = C::rad(p), nb = (C::E / r) * (r - 1);
    if (i < nb) {
      const int b = i / (r - 1), q = i % (r - 1) + 1;
      const int k = (t + b * C::T) & (ns - 1);
      return q * k * (1024 / (ns * r));
    }
    i -= nb;
    ns *= r;
  }
  return 0;
}

// Lane-major copies of the register twiddles, stored after the W_1024 table:
// lane t of size N reads tw_pad<N>() consecutive values (an even count, so the
// rows are 16-byte aligned) starting at twl_off(N) + t tw_pad<N>().
template <int N>
__host__ __device__ constexpr int tw_pad() { return (tw_count<N>() + 1) & ~1; }
__host__ __device__ constexpr int twl_off(int n) {
  int o = 1024;
  if (n > 64) o += FftCfg<64>::T * tw_pad<64>();
  if (n > 128) o += FftCfg<128>::T * tw_pad<128>();
  if (n > 256) o += FftCfg<256>::T * tw_pad<256>();
  if (n > 512) o += FftCfg<512>::T * tw_pad<512>();
  return o;
}
constexpr int kTwTotal = twl_off(1024) + FftCfg<1024>::T * tw_pad<1024>();

// tab: W_1024^m = exp(-2 pi i m / 1024), m in [0, 1024), followed by the
// lane-major copies (global memory).
template <int N>
__device__ __forceinline__ void tw_load(Twiddles<N>& tw, int t, const float2* __restrict__ tab) {
  constexpr int TC = tw_count<N>(), TP = tw_pad<N>();
  const float4* row = reinterpret_cast<const float4*>(tab + twl_off(N) + t * TP);
#pragma unroll
  for (int i = 0; i < TP / 2; ++i) {
    const float4 v = row[i];
    tw.w[2 * i] = make_float2(v.x, v.y);
    if (2 * i + 1 < TC) tw.w[2 * i + 1] = make_float2(v.z, v.w);
  }
}

// ---------------------------------------------------------------- Stockham pass
// Where a transform's scratch element i lives: ExchIdx of a private row (the
// default), or row col_swz(i) of a column of a larger LDS array whose rows
// are `stride` complex values apart.  col_swz permutes the rows within the
// column (XOR of the low bits with a function of the high bits) so that the
// T lanes of an FFT group hit T different banks in every exchange of the
// Stockham passes, including the first pass's writes 8 elements apart, which
// a plain strided column sends to one or two banks.
template <int N> __device__ __forceinline__ int col_swz(int i);
template <> __device__ __forceinline__ int col_swz<64>(int i) { return i ^ ((i >> 3) & 7); }
template <> __device__ __forceinline__ int col_swz<128>(int i) { return i ^ (((i >> 4) + ((i >> 6) << 3)) & 15); }

// Exchange layouts of a private scratch row, per pass (N >= 256).  On this
// LDS an 8-byte read serves 32 lanes per cycle over 64 banks, an 8-byte write
// 16 lanes over 32 banks.  After pass 0 (writes 8t + q or 16t + q, reads
// t + e T) i + i/16 keeps the writes conflict-free, at the price of a 2-way
// conflict on the reads (the cheaper of the two: a write takes twice the
// cycles of a read).  After pass 1 a lane writes the NS1 = rad(0) consecutive
// elements of a block of NS1 rad(1) at stride NS1, and the lanes of a cycle
// span several such blocks, which a padding of one slot per 16 or 32 sends to
// the same banks; shifting block b by NS1 b makes both the writes and the
// reads conflict-free.  Below 256 (several transforms per wavefront) lidx
// serves both exchanges.
template <int N>
struct ExchIdx {
  template <int P>
  __device__ __forceinline__ int at(int i) const {
    if constexpr (N < 256) {
      return lidx(i);
    } else if constexpr (P == 0) {
      return i + (i >> 4);
    } else {
      constexpr int NS1 = FftCfg<N>::rad(0), BL = NS1 * FftCfg<N>::rad(1);
      return i + NS1 * (i / BL);
    }
  }
};
// Scratch elements a transform needs in its private row: the callers' lidx
// layout and every exchange layout.
template <int N>
__host__ __device__ constexpr int fft_scratch() {
  const int a = lidx(N - 1) + 1;
  if (N < 256) return a;
  const int NS1 = FftCfg<N>::rad(0), BL = NS1 * FftCfg<N>::rad(1);
  const int b = (N - 1) + NS1 * ((N - 1) / BL) + 1, c = (N - 1) + ((N - 1) >> 4) + 1;
  const int m = a > b ? a : b;
  return m > c ? m : c;
}
template <int N>
struct ColumnIdx {
  int stride;
  template <int P>
  __device__ __forceinline__ int at(int i) const {
    return col_swz<N>(i) * stride;
  }
};

// REG: twiddles from registers (twr), otherwise loaded from the table per pass.
template <int N, bool INV, int P, int NS, bool REG, class IX = ExchIdx<N>>
__device__ __forceinline__ void fft_pass(float2 (&v)[FftCfg<N>::E], float2* __restrict__ lds, int t,
                                         const Twiddles<N>* __restrict__ twr, const float2* __restrict__ tab,
                                         IX ix = IX()) {
  using C = FftCfg<N>;
  constexpr int R = C::rad(P), E = C::E, T = C::T, B = E / R;
  constexpr bool LAST = (P == C::NP - 1);
  constexpr int TWS = 1024 / (NS * R);
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int j = t + b * T;
    const int k = j & (NS - 1);
    float2 u[R];
#pragma unroll
    for (int q = 0; q < R; ++q) u[q] = v[b + q * B];
    if constexpr (P > 0) {
#pragma unroll
      for (int q = 1; q < R; ++q) {
        float2 w;
        if constexpr (REG) w = twr->w[tw_off<N>(P) + b * (R - 1) + q - 1];
        else w = tab[q * k * TWS];
        if (INV) w.y = -w.y;
        u[q] = cmul(u[q], w);
      }
    }
    Dft<R, INV>::run(u);
    if constexpr (LAST) {
#pragma unroll
      for (int q = 0; q < R; ++q) v[b + q * B] = u[q];
    } else {
      const int base = (j / NS) * NS * R + k;
#pragma unroll
      for (int q = 0; q < R; ++q) lds[ix.template at<P>(base + q * NS)] = u[q];
    }
  }
  if constexpr (!LAST) {
    wave_lds_sync();
#pragma unroll
    for (int e = 0; e < E; ++e) v[e] = lds[ix.template at<P>(t + e * T)];
    wave_lds_sync();
    fft_pass<N, INV, P + 1, NS * R, REG, IX>(v, lds, t, twr, tab, ix);
  }
}

// Full transform with register twiddles.  lds: this transform's private
// scratch of fft_scratch<N>() float2.  Forward: X[k] = sum_n x[n] exp(-2 pi i k n / N);
// inverse: exp(+...), unscaled.
template <int N, bool INV>
__device__ __forceinline__ void fft_wave(float2 (&v)[FftCfg<N>::E], float2* __restrict__ lds, int t,
                                         const Twiddles<N>& tw) {
  fft_pass<N, INV, 0, 1, true>(v, lds, t, &tw, nullptr);
}

// Full transform with register twiddles whose scratch is a column of a
// larger LDS array: element i of the scratch at lds[col_swz<N>(i) * stride]
// (N = 64, 128).
// The lane index goes through an empty asm statement so that each call
// recomputes its scratch addresses instead of keeping those of earlier calls
// live in registers.
template <int N, bool INV>
__device__ __forceinline__ void fft_wave_column(float2 (&v)[FftCfg<N>::E], float2* __restrict__ lds, int t,
                                                const Twiddles<N>& tw, int stride) {
  int tl = t;
  asm volatile("" : "+v"(tl));
  fft_pass<N, INV, 0, 1, true, ColumnIdx<N>>(v, lds, tl, &tw, nullptr, ColumnIdx<N>{stride});
}

// Same, reading twiddles from the W_1024 table in every pass.
template <int N, bool INV>
__device__ __forceinline__ void fft_wave_tab(float2 (&v)[FftCfg<N>::E], float2* __restrict__ lds, int t,
                                             const float2* __restrict__ tab) {
  fft_pass<N, INV, 0, 1, false>(v, lds, t, nullptr, tab);
}

}  // namespace swift
