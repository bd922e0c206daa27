// Internal declarations shared by the kernel sources and the C ABI layer.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/swift.h"

namespace swift {

constexpr float kNearTieRel = 2e-4f;
// A window is degenerate when its taper-weighted variance ||w||^2 is at most
// this fraction of the energy of its samples about the offset (sum (a'T)^2):
// its samples are then equal up to rounding.
constexpr double kDegenerateRel = 1e-6;

// Every sample a of a window is taken about an offset o, a' = a - o: the
// source pixel nearest the window centre, read alike by every block of the
// pair.  The weighted mean is removed exactly in the frequency domain
// afterwards, so the offset changes nothing mathematically; it keeps the sums
// of low-contrast windows with large values free of cancellation, and makes
// the samples of a constant window exactly zero.
//
// Per row-slice partial sums of the forward row pass (A then B):
// s[0] = sum a'T, s[1] = sum (a'T)^2, s[2] = sum a'T^2.
struct RowPart {
  double s[6];
  int32_t clamped;
  float off[2];   // oA, oB (the same in every slice of a pair)
  int32_t pad;
};

// Per pair, after reducing the row partials.  The cross power is formed from
// the normalised spectra F_A / ||w_A|| and F_B / ||w_B||, so that |X|^2 stays
// in FP32 range for any input scale; kw restores the surface's scale.
struct PairStat {
  float mA, mB;   // taper-weighted means of the offset samples a - oA, b - oB
  float oA, oB;   // the offsets
  float sA, sB;   // 1 / ||w_A||, 1 / ||w_B|| (0 for a degenerate pair)
  float swA, swB; // ||w_A||^2, ||w_B||^2
  float kw;       // (||w_A|| ||w_B||)^(1-p) / N^2 (0 for a degenerate pair)
  int32_t flags;  // bit 0: degenerate (a window is constant); bit 2: clamped
  int32_t pad[2];
};

// Per pair and image, computed once per pair before the forward row pass:
// the window's origin split into integer and fractional parts, whether its
// linear part is the identity, and its offset (the centre pixel).
struct WinGeom {
  int32_t bx0, by0;  // floor(cx + tx), floor(cy + ty) (clamped to +-1e9)
  float fx, fy;      // the fractional parts
  float off;         // img[clamp(floor(y + 1/2))][clamp(floor(x + 1/2))]
  int32_t flags;     // bit 0: translation window; bit 1: origin within +-1e8
};
struct PairGeom {
  WinGeom w[2];      // A, B
};

// Per row-slice partials of the inverse row pass.
struct InvPart {
  float m1;       // largest value
  int32_t i1;     // its flat index (smallest on ties)
  float m2;       // largest value elsewhere
  int32_t pad;
  double sum, sumsq;
};

// Taper spectrum of one window size: tau[k] = sum_i t(i) exp(-2 pi i k i / N)
struct TaperInfo {
  double sum_t, sum_t2;
  int32_t L;
  int32_t pad;
};

struct MatchArgs {
  const swift_image* imgs;
  const int32_t* img_a;
  const int32_t* img_b;
  const float* th_a;
  const float* th_b;
  swift_match* out;
  float* surfaces;      // NULL or this group's first surface
  float2* Z;            // [P][N][N] exchange buffer
  RowPart* rowpart;     // [P][NSLICE]
  PairStat* pstat;      // [P]
  InvPart* invpart;     // [P][NSL2]
  PairGeom* geom;       // [P]
  const float2* tw;     // W_1024 table
  const float2* tau;    // [N]
  const float* taper;   // [N] t(i)
  const TaperInfo* tinfo;
  float p, eps_rel;
  int32_t L;            // taper samples per edge
  int32_t snr_exclude_r;  // R > 0: the SNR background leaves out the (2R+1)^2 box at the peak
  int32_t npairs;
  int32_t nsl_fwd, nsl_inv;  // row blocks per pair of the forward / inverse row passes
  int32_t n_imgs;
  // Pruned inverse (max_shift = r > 0): the peak is searched among wrapped
  // shifts |sx|, |sy| <= r; the column pass stores surface rows [0, zlo) and
  // [zhi, N) only, which the inverse row pass covers with its first nsl_lo
  // row blocks and its last nsl_inv - nsl_lo (nsl_inv counts the launched
  // blocks); colsq [P][N/2+1] receives the column sums of |C|^2 (Hermitian
  // weights) that give the background std by Parseval.  Unpruned: r = 0,
  // zlo = zhi = N, nsl_lo = nsl_inv.
  int32_t max_shift, zlo, zhi, nsl_lo;
  double* colsq;
  // Pearson mode (max_shift = N/4, p = 0, box taper tables): ncc_rows
  // [P][N][N/2+1] holds window B's row sums (f', f'^2) over the template
  // width at every placement, ncc_var [P][N/2+1][N/2+1] the patch energy
  // sum (f - mean)^2 of every placement.
  int32_t pearson;
  float2* ncc_rows;
  float* ncc_var;
  // state kept for the adjoint (all NULL when not requested)
  float2* saved_Z;         // [P][N][N]: forward 2-D spectrum of z, [kx][ky]
  PairStat* saved_ps;      // [P]
  swift_match* saved_rec;  // [P]
  float* saved_nb;         // [P][9] surface values around the peak ([dy+1][dx+1])
};

// Arguments of the adjoint kernels of one window size.
struct BwdArgs {
  const swift_image* imgs;
  const int32_t* img_a;
  const int32_t* img_b;
  const float* th_a;
  const float* th_b;
  const float2* Zf;         // saved forward spectrum [P][kx][ky]
  const PairStat* ps;       // saved
  const swift_match* rec;   // saved
  const float* nb;          // saved [P][9]
  const float* g_peak;      // [P] or NULL
  const float* g_snr;       // [P] or NULL
  float* g_th_a;            // [P][6]
  float* g_th_b;            // [P][6] or NULL
  float2* Y;                // [P][kx][y] inverse-column output
  double* dpart;            // [P][NW][kDpart] partial dJ/d(eps^2) (two objectives) and Hessian sums
  float* peak_hess;         // [P][3] or NULL
  float* jac;               // [P][2][6] (centroid-Jacobian mode)
  double* rpart;            // [P][NSLICE][40] partial pixel sums
  const float2* tw;
  const float2* tau;
  const float* taper;
  const TaperInfo* tinfo;
  float p, eps_rel;
  int32_t L;
  int32_t npairs;
  int32_t n_imgs;
  int32_t jac_trans;  // centroid-Jacobian mode: translation columns only
};
constexpr int kBwdSums = 20;  // per image: P1[6], P2[6], P3[6], Q, R
constexpr int kDpart = 6;     // dJ0/de2, dJ1/de2, hxx, hyy, hxy, unused

// Rows per block of the row passes, per window size.  FWD: forward row pass
// (and adjoint row pass); INV: inverse row pass; TILE: LDS bytes of the uint8
// source tile of a forward block (0: gather straight from memory); TRW:
// 16-byte tile loads per thread (each wave load covers 64 / tile_cw<N> tile
// rows).  FWD2 / INV2 (with TILE2, TRW2) are the alternative row counts
// swift_autotune can choose; the defaults are FWD / INV.
template <int N> struct RowsCfg;
template <> struct RowsCfg<64>   { static constexpr int FWD = 32, INV = 64, TILE = 4608,  TRW = 2,
                                   FWD2 = 32, INV2 = 32, TILE2 = 4608, TRW2 = 2; };
template <> struct RowsCfg<128>  { static constexpr int FWD = 16, INV = 32, TILE = 6144,  TRW = 2,
                                   FWD2 = 32, INV2 = 64, TILE2 = 8960, TRW2 = 3; };
template <> struct RowsCfg<256>  { static constexpr int FWD = 16, INV = 16, TILE = 9728,  TRW = 4,
                                   FWD2 = 8,  INV2 = 32, TILE2 = 5632, TRW2 = 3; };
template <> struct RowsCfg<512>  { static constexpr int FWD = 8,  INV = 16, TILE = 11264, TRW = 5,
                                   FWD2 = 4,  INV2 = 8,  TILE2 = 8576, TRW2 = 4; };
template <> struct RowsCfg<1024> { static constexpr int FWD = 8,  INV = 16, TILE = 24576, TRW = 6,
                                   FWD2 = 4,  INV2 = 8,  TILE2 = 16384, TRW2 = 4; };

// Rows per workgroup of the adjoint's row pass, its uint8 tile budget and
// tile loads per thread.  The pass keeps the stage and the tile in separate
// LDS arrays; at 1024^2 it takes four rows, so that both fit three
// workgroups per CU; otherwise the forward row pass's defaults.
template <int N> struct BwdRowsCfg {
  static constexpr int R = N >= 1024 ? RowsCfg<N>::FWD2 : RowsCfg<N>::FWD;
  static constexpr int TILE = N >= 1024 ? RowsCfg<N>::TILE2 : RowsCfg<N>::TILE;
  static constexpr int TRW = N >= 1024 ? RowsCfg<N>::TRW2 : RowsCfg<N>::TRW;
};

constexpr int kSizes[SWIFT_NSIZES] = {64, 128, 256, 512, 1024};

size_t align256(size_t x);

// Optional kernel timing: when non-null, launchers bracket every kernel with
// begin/end so the context can record HIP events on the launch stream.
struct KernelTimer {
  virtual void begin(const char* name, int n, hipStream_t s) = 0;
  virtual void end(hipStream_t s) = 0;
  virtual ~KernelTimer() {}
};

// Launchers (return hipError_t of the launch).
// box = true: the Pearson tables (unit gather taper, tau = DFT of the central
// n/2 template box, box sums).
hipError_t launch_taper(int n, float taper_frac, float2* tau, float* taper, TaperInfo* info, hipStream_t s,
                        bool box = false);
// fwd_variant 0 / 1 and alt_inv select the row counts of the five-kernel
// path (FWD / FWD2, INV / INV2; the slice counts a.nsl_fwd and a.nsl_inv must
// match the choice).  fwd_variant 2 (n <= kFusedMaxN, not Pearson) runs the
// whole pair in one workgroup (launch_fused_group).
constexpr int kFusedVariant = 2;
constexpr int kFusedMaxN = 128;
hipError_t launch_match_group(int n, const MatchArgs& a, int fwd_variant, bool alt_inv, hipStream_t s, KernelTimer* kt);
hipError_t launch_fused_group(int n, const MatchArgs& a, hipStream_t s, KernelTimer* kt);
int fwd_blocks_n(int n, bool alt);  // forward row blocks per pair
int inv_blocks_n(int n, bool alt);  // inverse row blocks per pair
hipError_t launch_backward_group(int n, const BwdArgs& a, bool centroid_jac, hipStream_t s, KernelTimer* kt);
int bwd_col_blocks_n(int n);  // adjoint column-stage workgroups per pair
int bwd_row_blocks_n(int n);  // adjoint row-stage workgroups (row slices) per pair
hipError_t launch_snr(const float* surf, int n, int batch, int exclude_r, swift_match* out, hipStream_t s);
hipError_t launch_render(const uint8_t* src, int64_t spitch, int64_t sstride, int S, int sh, int sw,
                         const double* aff, int level, uint8_t* dst, int64_t dpitch, int64_t dstride, int dh, int dw,
                         hipStream_t st, KernelTimer* kt);
hipError_t launch_render_mesh(const uint8_t* src, int64_t spitch, int64_t sstride, int S, int sh, int sw,
                              const double* tri_aff, int grid, int level, uint8_t* dst, int64_t dpitch,
                              int64_t dstride, int dh, int dw, hipStream_t st, KernelTimer* kt);
// mesh: aff holds per-triangle affines [S][2 (grid-1)^2][6] instead of [S][6]
hipError_t launch_stack_windows(int S, const double* aff, int level, int grid, int hl, int wl, int img_a0,
                                int img_b0, float* th_a, float* th_b, int32_t* ia, int32_t* ib, bool mesh,
                                hipStream_t st);
hipError_t launch_fit_sections(int S, int per, const float* th_a, const float* th_b, const swift_match* rec,
                               int level, float min_snr, double* aff, int32_t* status, hipStream_t st);
hipError_t launch_fit_mesh(int S, int grid, const float* th_a, const float* th_b, const swift_match* rec, int level,
                           float min_snr, const double* aff, double* tri_aff, int32_t* status, hipStream_t st,
                           KernelTimer* kt);
hipError_t launch_refine(int P, const swift_match* rec, const float* jac, float* th, int mode, float max_step,
                         float* step_out, hipStream_t s);
// side 0: two-sided model; -1 / +1: one-sided (sections before / after).
hipError_t launch_project(const uint8_t* src, int64_t pitch, int64_t sstride, int S, int H, int W,
                          const uint8_t* exclude, int k, uint8_t* dst, int64_t dpitch, int64_t dstride,
                          hipStream_t s, KernelTimer* kt, int side = 0);
hipError_t launch_blend_span(int a, int b, const double* left, const double* right, double* aff, hipStream_t st);
hipError_t launch_join_break(int S, int j, const double* in, const double* left, double* out, hipStream_t st);
hipError_t launch_search_next(int P, const uint8_t* done, float ox, float oy, const int32_t* img_a,
                              const int32_t* img_b, const float* theta_a, const float* theta_b, int32_t* idx,
                              int32_t* ia, int32_t* ib, float* ta, float* tb, int32_t* count, hipStream_t st);
hipError_t launch_search_keep(int P, int n, const int32_t* idx, const swift_match* recs, int cand, float accept,
                              swift_match* best, int32_t* best_cand, uint8_t* done, hipStream_t st);
hipError_t launch_pyramid(const uint8_t* src, int64_t spitch, int sw, int sh, uint8_t* dst, int64_t dpitch,
                          int dw, int dh, hipStream_t s);

}  // namespace swift
