// Pair kernel with the coordinate cross term on the matrix cores (GP_BF16X): for float inputs
// and d <= 64,
//   rho_ij = n_i + n_j - 2 x~_i . x~_j
// with x~ split into bfloat16 hi + lo (truncation; |x - hi - lo| <= 2^-16 |x|), the cross term
// formed by v_mfma_f32_16x16x32_bf16 from three products (hi.hi + hi.lo + lo.hi) and the
// compensated norms n_i = sum_k (h_ik^2 + 2 h_ik l_ik) computed in double from the same parts,
// so rho_ij = |x_i - x_j|^2 - |l_i - l_j|^2 (the dropped lo.lo terms cancel on the diagonal and
// leave an error relative to the distance itself) up to float accumulation.  rho is clamped at 0.
// K Y takes K rounded to the nearest float16 times Y hi + lo (two products) with the diagonal
// pairs left out and alpha y_i added in double in the epilogue, so the large diagonal is exact
// and the zero-mean rounding of the other entries stays far inside the bfloat16 budget.  The
// quad weights S, which only the length-scale gradient uses (through W off the diagonal), take
// Q rounded to the nearest float16 times P hi + lo (two products, the same argument).  For the
// per-coordinate (ARD) gradient the identity
//   sum_ij W_ij (x_ik - x_jk)^2 = sum_i [ x_ik^2 (W 1)_i + (W X^2)_ik - 2 x_ik (W X)_ik ]
// turns the d sums into one more MFMA product W [X | X^2 | 1]: W rounded to the nearest
// bfloat16 and [X | X^2 | 1] split hi/lo, two products.  The same rounded W multiplies every
// column, so the identity holds exactly for it and its zero-mean rounding averages out of the
// sums instead of being amplified by the cancellation between the three terms.
// Layouts are those of pair_mfma.hip: lane l = 16 g + m; A[m][8g + q], B[8g + q][m],
// D[4g + r][m]; the k index of the products over j runs in the slot order 8g + q <-> j =
// 16 (q / 4) + 4 g + (q % 4).
#include "pass.h"

namespace gpk {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __fp16 f16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
typedef _Float16 h16x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

namespace xm {

constexpr int kWaves = 8;
constexpr int kWG = kWaves * 64;
constexpr int TJ = 32;           // columns per tile
constexpr int kStrideH = 40;     // halves per LDS row of the 32-wide operands
constexpr int kFold = 8;         // tiles between folds of the float partials
constexpr int kScaleTop = 14;
constexpr int kAmaxBlocks = 64;

union H8 {
  f16x8 v;
  uint32_t u[4];
};
union B8 {
  bf16x8 v;
  uint32_t u[4];
  uint16_t h[8];
};

__device__ __forceinline__ uint32_t pk_rtz(float a, float b) {
  f16x2 h = __builtin_amdgcn_cvt_pkrtz(a, b);
  return __builtin_bit_cast(uint32_t, h);
}
__device__ __forceinline__ void split16(float x, float &hi, float &lo) {
  hi = __uint_as_float(__float_as_uint(x) & 0xFFFFE000u);
  lo = x - hi;
}
// bfloat16 hi/lo by truncation: hi = top 16 bits of x, lo = top 16 bits of x - hi
__device__ __forceinline__ void splitbf(float x, uint16_t &hb, uint16_t &lb) {
  const uint32_t b = __float_as_uint(x);
  hb = (uint16_t)(b >> 16);
  const float l = x - __uint_as_float(b & 0xFFFF0000u);
  lb = (uint16_t)(__float_as_uint(l) >> 16);
}
__device__ __forceinline__ float bfval(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// A 32-column tile as stage_tiles_xm lays it out in global memory, byte for byte the image of one
// LDS tile buffer: bf16 coordinates hi and lo (a padded row of DPX values per point), the norms,
// with the gradient Q (float16, a padded row of 32 halves per point, c >= RP zero), Y^T hi and lo
// (a padded row of 32 slot-ordered halves per column c), and for the per-coordinate gradient the
// bf16 hi and lo of [X | X^2 | 1]^T (a padded row of 32 slot-ordered values per k2), rounded up
// to whole 1 KB wave copies.  Every region is a multiple of 16 bytes.
template <int DPX, int RP, int GM>
struct XTile {
  static constexpr int XSTR = DPX + 8;
  static constexpr int KB2 = GM == 2 ? (2 * DPX + 16) / 16 : 0;
  static constexpr int kXB = TJ * XSTR * 2;
  static constexpr int kNB = TJ * 4;
  static constexpr int kQB = GM ? TJ * kStrideH * 2 : 0;
  static constexpr int kYB = RP * kStrideH * 2;
  static constexpr int kBB = KB2 * 16 * kStrideH * 2;
  static constexpr int kOffXL = kXB;
  static constexpr int kOffN = 2 * kXB;
  static constexpr int kOffQH = kOffN + kNB;
  static constexpr int kOffYH = kOffQH + kQB;
  static constexpr int kOffYL = kOffYH + kYB;
  static constexpr int kOffBH = kOffYL + kYB;
  static constexpr int kOffBL = kOffBH + kBB;
  static constexpr int kBytes = (kOffBL + kBB + 1023) / 1024 * 1024;
};

struct XArgs {
  int64_t n;
  int R, L, d;
  const float *xs;  // n x xst scaled coordinates (float)
  int xst;
  const uint16_t *xh, *xl;  // n x DPX bf16 hi / lo
  const float *nrm;         // n norms of hi + lo
  const double *theta;
  const float *Y;
  int64_t ldy;
  const float *P;
  int64_t ldp;
  const float *Q;
  int64_t ldq;
  const double *w;
  const float *D;
  int64_t ldd;
  const double *col_shift;
  int no_noise;
  float *out;
  int64_t ldo;
  int64_t col_chunk;
  int splits;
  double *outp;
  double *rec;
  int nth, nrec;
  const int *scl;
  float *amax;
  u32x4 *stage;  // column tiles laid out by stage_tiles_xm
};

// hi/lo bf16 coordinates (zero-padded to dpx) and their compensated norms, one point per thread
__global__ __launch_bounds__(256) void xm_prep(const float *xs, int64_t n, int xst, int dpx,
                                               uint16_t *xh, uint16_t *xl, float *nrm) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int k = 0; k < dpx; ++k) {
    const float x = k < xst ? xs[i * xst + k] : 0.0f;
    uint16_t hb, lb;
    splitbf(x, hb, lb);
    xh[i * dpx + k] = hb;
    xl[i * dpx + k] = lb;
    // compensated norm: the terms h^2 + 2 h l that the three cross-term products form, so the
    // diagonal gets rho = 0 and rho_ij = |x_i - x_j|^2 - |l_i - l_j|^2 exactly in exact arithmetic
    const double h = (double)bfval(hb), l = (double)bfval(lb);
    s += h * h + 2.0 * h * l;
  }
  nrm[i] = (float)s;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  return v;
}

__global__ __launch_bounds__(256) void absmax_partial(XArgs a) {
  __shared__ float sh[4];
  const int which = blockIdx.y;
  const float *A = which == 0 ? a.Y : (which == 1 ? a.P : a.Q);
  const int64_t ld = which == 0 ? a.ldy : (which == 1 ? a.ldp : a.ldq);
  float m = 0.0f;
  if (A) {
    const int64_t ne = a.n * a.R;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < ne; e += (int64_t)gridDim.x * 256) {
      const int64_t i = e / a.R;
      const int c = (int)(e - i * a.R);
      float v = fabsf(A[i * ld + c]);
      if (which == 1 && a.w) v = fabsf((float)((double)A[i * ld + c] * a.w[c]));
      m = fmaxf(m, v);
    }
  }
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0)
    a.amax[which * kAmaxBlocks + blockIdx.x] = fmaxf(fmaxf(sh[0], sh[1]), fmaxf(sh[2], sh[3]));
}

__device__ int scale_exp(float m) {
  if (!(m > 0.0f) || !isfinite(m)) return 0;
  int e;
  frexpf(m, &e);
  e = kScaleTop - e;
  return e > 100 ? 100 : (e < -100 ? -100 : e);
}

__global__ void scales_final(XArgs a, int *scl) {
  if (threadIdx.x != 0) return;
  int eK = kScaleTop - (int)ceil(a.theta[0] * kLog2e);
  eK = eK > 100 ? 100 : (eK < -100 ? -100 : eK);
  scl[0] = eK;
  for (int which = 0; which < 3; ++which) {
    float m = 0.0f;
    for (int b = 0; b < kAmaxBlocks; ++b) m = fmaxf(m, a.amax[which * kAmaxBlocks + b]);
    scl[1 + which] = scale_exp(m);
  }
}

// Split, scale and lay out the column side of every 32-column tile as the LDS image of XTile.
// Columns past n get zero operands, a huge norm (their kernel values vanish) and no ones entry.
template <int DPX, int RP, int GM>
__global__ __launch_bounds__(256) void stage_tiles_xm(XArgs a, int64_t ntiles) {
  using G = XTile<DPX, RP, GM>;
  constexpr int kCh = G::kBytes / 16;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= ntiles * kCh) return;
  const int64_t tile = e / kCh;
  const int off = 16 * (int)(e - tile * kCh);
  const int64_t jt = tile * TJ;
  union {
    u32x4 v;
    _Float16 h[8];
    uint16_t u[8];
    float f[4];
  } out;
  out.v = u32x4{0u, 0u, 0u, 0u};
  // column of slot sl in the slot order of the products over j
  auto slot_col = [](int sl) { return 16 * ((sl & 7) >> 2) + 4 * (sl >> 3) + (sl & 3); };
  if (off < G::kOffN) {
    const bool lo = off >= G::kOffXL;
    const int o = off - (lo ? G::kOffXL : 0);
    const int jj = o / (2 * G::XSTR), k0 = (o - jj * 2 * G::XSTR) / 2;
    const int64_t j = jt + jj;
    if (k0 < DPX && j < a.n) out.v = *(const u32x4 *)&(lo ? a.xl : a.xh)[j * DPX + k0];
  } else if (off < G::kOffQH) {
    const int jj0 = (off - G::kOffN) / 4;
#pragma unroll
    for (int u = 0; u < 4; ++u) out.f[u] = jt + jj0 + u < a.n ? a.nrm[jt + jj0 + u] : 1.0e30f;
  } else if (off < G::kOffYH) {
    const int o = off - G::kOffQH;
    const int jj = o / (2 * kStrideH), c0 = (o - jj * 2 * kStrideH) / 2;
    const int64_t j = jt + jj;
    const float sQ = ldexpf(1.0f, a.scl[3]);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int c = c0 + u;
      // rounded to nearest (the float16 conversion's mode)
      out.h[u] = (_Float16)((j < a.n && c < RP && c < a.R) ? a.Q[j * a.ldq + c] * sQ : 0.0f);
    }
  } else if (off < G::kOffBH) {
    const bool lo = off >= G::kOffYL;
    const int o = off - (lo ? G::kOffYL : G::kOffYH);
    const int c = o / (2 * kStrideH), s0 = (o - c * 2 * kStrideH) / 2;
    const float sY = ldexpf(1.0f, a.scl[1]);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int sl = s0 + u;
      const int64_t j = jt + (sl < 32 ? slot_col(sl) : 0);
      float h, l;
      split16((sl < 32 && j < a.n && c < a.R) ? a.Y[j * a.ldy + c] * sY : 0.0f, h, l);
      out.h[u] = (_Float16)(lo ? l : h);
    }
  } else if (GM == 2 && off < G::kOffBL + G::kBB) {
    const bool lo = off >= G::kOffBL;
    const int o = off - (lo ? G::kOffBL : G::kOffBH);
    const int k2 = o / (2 * kStrideH), s0 = (o - k2 * 2 * kStrideH) / 2;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int sl = s0 + u;
      const int64_t j = jt + (sl < 32 ? slot_col(sl) : 0);
      uint16_t hb = 0, lb = 0;
      if (sl < 32 && j < a.n) {
        if (k2 < 2 * DPX) {
          const int k = k2 < DPX ? k2 : k2 - DPX;
          const float x = k < a.xst ? a.xs[j * a.xst + k] : 0.0f;
          splitbf(k2 < DPX ? x : x * x, hb, lb);
        } else if (k2 == 2 * DPX) {
          hb = 0x3F80;  // 1.0
        }
      }
      out.u[u] = lo ? lb : hb;
    }
  }
  a.stage[e] = out.v;
}

// DPX: padded coordinate width of the cross term (32 or 64).  RP: padded R (16 or 32).
// GM: 0 product only, 1 isotropic gradient, 2 per-coordinate gradient.  IB: row blocks / wave.
template <int DPX, int RP, int GM, int IB>
__global__ __launch_bounds__(kWG) void pair_xm(XArgs a) {
  constexpr int KC = DPX / 32;               // k chunks of the cross term
  constexpr int NCB = RP / 16;
  constexpr int KB2 = GM == 2 ? (2 * DPX + 16) / 16 : 1;  // blocks of [X | X^2 | 1]
  constexpr int XSTR = DPX + 8;              // halves per LDS row of the coordinate tile
  constexpr int kRowsWG = kWaves * IB * 16;
  using XT = XTile<DPX, RP, GM>;
  __shared__ __attribute__((aligned(16))) char tile0[XT::kBytes];
  __shared__ __attribute__((aligned(16))) char tile1[XT::kBytes];
  __shared__ double shr[kWaves];
  __shared__ double sred[kWaves][64];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int m = lane & 15, g = lane >> 4;
  const int64_t row0 = (int64_t)blockIdx.x * kRowsWG + wave * (IB * 16);
  const int R = a.R;
  const int eK = a.scl[0], eY = a.scl[1], eP = a.scl[2], eQ = a.scl[3];
  const float c0 = (float)(a.theta[0] * kLog2e + (double)eK);

  // ---- row side ----------------------------------------------------------------------------
  B8 xbh[IB][KC], xbl[IB][KC];
  float ai[IB];
  H8 ph[IB], pl[IB];
  float xr[IB][4][GM == 2 ? DPX / 16 : 1];  // x~[16 ib + 4 g + r][16 kb + m]
#pragma unroll
  for (int ib = 0; ib < IB; ++ib) {
    int64_t i = row0 + ib * 16 + m;
    const bool row_ok = i < a.n;
    if (!row_ok) i = a.n - 1;
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
      xbh[ib][kc].v = *(const bf16x8 *)&a.xh[i * DPX + 32 * kc + 8 * g];
      xbl[ib][kc].v = *(const bf16x8 *)&a.xl[i * DPX + 32 * kc + 8 * g];
    }
    ai[ib] = c0 - a.nrm[i];
    if (GM) {
      const float sP = ldexpf(1.0f, eP);
      float v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int c = 8 * g + q;
        v[q] = (row_ok && c < R) ? (float)((double)a.P[i * a.ldp + c] * (a.w ? a.w[c] : 1.0)) * sP
                                 : 0.0f;
      }
#pragma unroll
      for (int q = 0; q < 8; q += 2) {
        float h0, l0, h1, l1;
        split16(v[q], h0, l0);
        split16(v[q + 1], h1, l1);
        ph[ib].u[q / 2] = pk_rtz(h0, h1);
        pl[ib].u[q / 2] = pk_rtz(l0, l1);
      }
    }
    if (GM == 2) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t ir = row0 + ib * 16 + 4 * g + r;
#pragma unroll
        for (int kb = 0; kb < DPX / 16; ++kb) {
          const int k = 16 * kb + m;
          xr[ib][r][kb] = (ir < a.n && k < a.xst) ? a.xs[ir * a.xst + k] : 0.0f;
        }
      }
    }
  }

  f32x4 acc[IB][NCB];
  double acc64[IB][NCB][4];
  f32x4 wx[IB][KB2];
  double G[GM == 2 ? DPX / 16 : 1];
  float gl = 0.0f;
  double gl64 = 0.0;
#pragma unroll
  for (int ib = 0; ib < IB; ++ib) {
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      acc[ib][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int r = 0; r < 4; ++r) acc64[ib][cb][r] = 0.0;
    }
#pragma unroll
    for (int kb = 0; kb < KB2; ++kb) wx[ib][kb] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
#pragma unroll
  for (int kb = 0; kb < (GM == 2 ? DPX / 16 : 1); ++kb) G[kb] = 0.0;
  const double unscale_out = ldexp(1.0, -(eK + eY));
  const double unscale_g = ldexp(1.0, -(eK + eP + eQ));

  const int64_t j0 = (int64_t)blockIdx.y * a.col_chunk;
  const int64_t j1 = j0 + a.col_chunk < a.n ? j0 + a.col_chunk : a.n;
  const int ntiles = (int)((j1 - j0 + TJ - 1) / TJ);

  // Column tiles are double-buffered: while tile t is computed from one LDS buffer, the waves
  // copy tile t + 1 (the image stage_tiles_xm wrote) straight into the other in 1 KB blocks and
  // wait for their copies only before the barrier that ends tile t.
  constexpr int kRounds = (XT::kBytes / 1024 + kWaves - 1) / kWaves;
  const char *gtiles = (const char *)a.stage + (j0 / TJ) * (int64_t)XT::kBytes + lane * 16;
  auto issue = [&](int t, char *dst) {
    const char *src = gtiles + (int64_t)t * XT::kBytes;
#pragma unroll
    for (int u = 0; u < kRounds; ++u) {
      const int off = (u * kWaves + wave) * 1024;
      if (off < XT::kBytes)
        __builtin_amdgcn_global_load_lds(src + off,
                                         (__attribute__((address_space(3))) void *)(dst + off),
                                         16, 0, 0);
    }
  };
  if (ntiles > 0) issue(0, tile0);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  // two tiles per loop trip, so that every LDS access names its buffer statically and the copies
  // into one buffer do not hold up the reads of the other
  auto tile_step = [&](int t, const char *cur, char *nxt) {
    if (t + 1 < ntiles) issue(t + 1, nxt);
    const uint16_t *sxh = (const uint16_t *)cur;
    const uint16_t *sxl = (const uint16_t *)(cur + XT::kOffXL);
    const float *snrm = (const float *)(cur + XT::kOffN);
    const _Float16 *sqh = (const _Float16 *)(cur + XT::kOffQH);
    const _Float16 *syh = (const _Float16 *)(cur + XT::kOffYH);
    const _Float16 *syl = (const _Float16 *)(cur + XT::kOffYL);
    const uint16_t *sbh = (const uint16_t *)(cur + XT::kOffBH);
    const uint16_t *sbl = (const uint16_t *)(cur + XT::kOffBL);
    // ---- cross term C^T[j][i] = x~_j . x~_i and quad weights S^T ---------------------------
    f32x4 C[IB][2], s[IB][2];
#pragma unroll
    for (int jb = 0; jb < 2; ++jb) {
#pragma unroll
      for (int ib = 0; ib < IB; ++ib) C[ib][jb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kc = 0; kc < KC; ++kc) {
        B8 ah, al;
        ah.v = *(const bf16x8 *)&sxh[(16 * jb + m) * XSTR + 32 * kc + 8 * g];
        al.v = *(const bf16x8 *)&sxl[(16 * jb + m) * XSTR + 32 * kc + 8 * g];
#pragma unroll
        for (int ib = 0; ib < IB; ++ib) {
          f32x4 z = C[ib][jb];
          z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah.v, xbh[ib][kc].v, z, 0, 0, 0);
          z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah.v, xbl[ib][kc].v, z, 0, 0, 0);
          z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al.v, xbh[ib][kc].v, z, 0, 0, 0);
          C[ib][jb] = z;
        }
      }
      if (GM) {
        H8 vh;
        vh.v = *(const f16x8 *)&sqh[(16 * jb + m) * kStrideH + 8 * g];
#pragma unroll
        for (int ib = 0; ib < IB; ++ib) {
          f32x4 z = {0.f, 0.f, 0.f, 0.f};
          z = __builtin_amdgcn_mfma_f32_16x16x32_f16(vh.v, ph[ib].v, z, 0, 0, 0);
          z = __builtin_amdgcn_mfma_f32_16x16x32_f16(vh.v, pl[ib].v, z, 0, 0, 0);
          s[ib][jb] = z;
        }
      }
    }
    // ---- kernel values and gradient weights (VALU) ------------------------------------------
    // The diagonal pairs are left out of the tile (K_ii = alpha enters in the epilogue): their
    // distance is exactly zero, but the expansion x_i^2 + x_j^2 - 2 x_i x_j gives it only to float
    // rounding, and the length-scale weights would cancel the large K_ii S_ii to that rounding.
    // `dtile` (wave-uniform) marks the tiles that hold a diagonal pair of this wave.
    const int64_t jt_cur = j0 + (int64_t)t * TJ;
    const bool dtile = jt_cur < row0 + IB * 16 && row0 < jt_cur + TJ;
    const int doff = dtile ? (int)(row0 - jt_cur) : 0;
    H8 kh[IB];
    B8 whb[IB];
#pragma unroll
    for (int jb = 0; jb < 2; ++jb) {
      float kv[IB][4], wv[IB][4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float nj = snrm[16 * jb + 4 * g + r];
#pragma unroll
        for (int ib = 0; ib < IB; ++ib) {
          float tt = fmaf(2.0f, C[ib][jb][r], ai[ib] - nj);
          tt = fminf(tt, c0);  // rho >= 0
          float kk = __builtin_amdgcn_exp2f(tt);
          if (dtile && 16 * ib + m + doff == 16 * jb + 4 * g + r) kk = 0.0f;
          kv[ib][r] = kk;
          if (GM) {
            const float W = kk * s[ib][jb][r];
            if (GM == 1) gl = fmaf(W, c0 - tt, gl);
            wv[ib][r] = W;
          }
        }
      }
#pragma unroll
      for (int ib = 0; ib < IB; ++ib) {
#pragma unroll
        for (int r = 0; r < 4; r += 2) {
          h16x2 kp;  // round to nearest
          kp[0] = (_Float16)kv[ib][r];
          kp[1] = (_Float16)kv[ib][r + 1];
          kh[ib].u[2 * jb + r / 2] = __builtin_bit_cast(uint32_t, kp);
          if (GM == 2) {
            bf16x2 wp;  // round to nearest
            wp[0] = (__bf16)wv[ib][r];
            wp[1] = (__bf16)wv[ib][r + 1];
            whb[ib].u[2 * jb + r / 2] = __builtin_bit_cast(uint32_t, wp);
          }
        }
      }
    }
    // ---- products: out += K Y, and W [X | X^2 | 1] ------------------------------------------
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      H8 yh, yl;
      yh.v = *(const f16x8 *)&syh[(16 * cb + m) * kStrideH + 8 * g];
      yl.v = *(const f16x8 *)&syl[(16 * cb + m) * kStrideH + 8 * g];
#pragma unroll
      for (int ib = 0; ib < IB; ++ib) {
        f32x4 z = acc[ib][cb];
        z = __builtin_amdgcn_mfma_f32_16x16x32_f16(kh[ib].v, yh.v, z, 0, 0, 0);
        z = __builtin_amdgcn_mfma_f32_16x16x32_f16(kh[ib].v, yl.v, z, 0, 0, 0);
        acc[ib][cb] = z;
      }
    }
    if (GM == 2) {
#pragma unroll
      for (int kb = 0; kb < KB2; ++kb) {
        B8 bh, bl;
        bh.v = *(const bf16x8 *)&sbh[(16 * kb + m) * kStrideH + 8 * g];
        bl.v = *(const bf16x8 *)&sbl[(16 * kb + m) * kStrideH + 8 * g];
#pragma unroll
        for (int ib = 0; ib < IB; ++ib) {
          f32x4 z = wx[ib][kb];
          z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(whb[ib].v, bh.v, z, 0, 0, 0);
          z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(whb[ib].v, bl.v, z, 0, 0, 0);
          wx[ib][kb] = z;
        }
      }
    }
    if ((t + 1) % kFold == 0 || t + 1 == ntiles) {
#pragma unroll
      for (int ib = 0; ib < IB; ++ib)
#pragma unroll
        for (int cb = 0; cb < NCB; ++cb) {
#pragma unroll
          for (int r = 0; r < 4; ++r) acc64[ib][cb][r] += (double)acc[ib][cb][r];
          acc[ib][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
      if (GM == 1) {
        gl64 += (double)gl;
        gl = 0.0f;
      }
      if (GM == 2) {
        // lane holds (W B)[i = 16 ib + 4 g + r][k2 = 16 kb + m]; the ones column (k2 = 2 DPX)
        // is in lane 16 g of block KB2 - 1
#pragma unroll
        for (int ib = 0; ib < IB; ++ib) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const float rs = __shfl(wx[ib][KB2 - 1][r], lane & ~15, 64);
#pragma unroll
            for (int kb = 0; kb < DPX / 16; ++kb) {
              const float x = xr[ib][r][kb];
              G[kb] += (double)(x * x * rs + wx[ib][kb + DPX / 16][r] - 2.0f * x * wx[ib][kb][r]);
            }
          }
#pragma unroll
          for (int kb = 0; kb < KB2; ++kb) wx[ib][kb] = f32x4{0.f, 0.f, 0.f, 0.f};
        }
      }
    }
    __builtin_amdgcn_s_waitcnt(0);  // this wave's copies of tile t + 1 have landed
    __syncthreads();
  };
  for (int t = 0; t < ntiles; t += 2) {
    tile_step(t, tile0, tile1);
    if (t + 1 < ntiles) tile_step(t + 1, tile1, tile0);
  }

  // ---- epilogue -----------------------------------------------------------------------------
  const int64_t blk = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
  double *rec = a.rec + blk * a.nrec;
  const double sigma2 = a.no_noise ? 0.0 : exp(a.theta[a.nth - 1]);
  const double alpha = exp(a.theta[0]);  // the diagonal kernel value, left out of the tiles
  double gA = 0.0, gS = 0.0;
  double qc[NCB];
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) qc[cb] = 0.0;
#pragma unroll
  for (int ib = 0; ib < IB; ++ib)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      const int c = 16 * cb + m;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = row0 + 16 * ib + 4 * g + r;
        if (i < a.n && c < R) {
          const double ky0 = acc64[ib][cb][r] * unscale_out;
          if (a.splits == 1) {
            const double yic = (double)a.Y[i * a.ldy + c];
            const double ky = ky0 + alpha * yic;
            const double v = ky + (sigma2 + (a.col_shift ? a.col_shift[c] : 0.0)) * yic;
            if (a.out) a.out[i * a.ldo + c] = (float)v;
            if (a.D) {
              const double dic = (double)a.D[i * a.ldd + c];
              qc[cb] += dic * v;
              if (GM) {
                const double wc = a.w ? a.w[c] : 1.0;
                gA += wc * dic * ky;
                gS += wc * (double)a.P[i * a.ldp + c] * (double)a.Q[i * a.ldq + c];
              }
            }
          } else {
            a.outp[((int64_t)blockIdx.y * a.n + i) * R + c] = ky0;
          }
        }
      }
    }
  gS *= sigma2;
  auto block_total = [&](double v) -> double {
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) shr[wave] = v;
    __syncthreads();
    double tot = 0.0;
    for (int w_ = 0; w_ < kWaves; ++w_) tot += shr[w_];
    return tot;
  };
  {
    const double tt = block_total(gA);
    if (tid == 0) rec[0] = tt;
  }
  if (GM == 2) {
    // per-coordinate sums: lanes sharing m hold k = 16 kb + m
#pragma unroll
    for (int kb = 0; kb < DPX / 16; ++kb) {
      double v = G[kb];
      v += __shfl_xor(v, 16, 64);
      v += __shfl_xor(v, 32, 64);
      __syncthreads();
      sred[wave][lane] = v;
      __syncthreads();
      if (tid < 16) {
        const int k = 16 * kb + tid;
        double tot = 0.0;
        for (int w_ = 0; w_ < kWaves; ++w_) tot += sred[w_][tid];
        if (k < a.L) rec[1 + k] = tot * unscale_g;
      }
    }
  } else {
    for (int k = 0; k < a.L; ++k) {
      const double tt = block_total(GM == 1 ? gl64 * unscale_g : 0.0);
      if (tid == 0) rec[1 + k] = tt;
    }
  }
  {
    const double tt = block_total(gS);
    if (tid == 0) rec[a.L + 1] = tt;
  }
#pragma unroll
  for (int cb = 0; cb < NCB; ++cb) {
    double v = qc[cb];
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    __syncthreads();
    sred[wave][lane] = v;
    __syncthreads();
    if (tid < 16) {
      const int c = 16 * cb + tid;
      double tot = 0.0;
      for (int w_ = 0; w_ < kWaves; ++w_) tot += sred[w_][tid];
      if (c < R) rec[a.nth + c] = tot;
    }
  }
}

// Column-split partials: as finalise_mfma in pair_mfma.hip.
__global__ __launch_bounds__(256) void finalise_xm(XArgs a, int has_grad) {
  __shared__ double sh4[4];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool live = i < a.n;
  const int R = a.R;
  const double sigma2 = a.no_noise ? 0.0 : exp(a.theta[a.nth - 1]);
  const double alpha = exp(a.theta[0]);  // the diagonal kernel value, left out of the tiles
  double *rec = a.rec + (int64_t)blockIdx.x * a.nrec;
  auto bsum = [&](double v) -> double {
    v = wave_sum(v);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh4[wid] = v;
    __syncthreads();
    return (sh4[0] + sh4[1]) + (sh4[2] + sh4[3]);
  };
  double gA = 0.0, gS = 0.0;
  for (int c = 0; c < R; ++c) {
    double q = 0.0;
    if (live) {
      double ky = 0.0;
      // the split partials in split order, 8 loads in flight
      for (int s0 = 0; s0 < a.splits; s0 += 8) {
        double t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u)
          t[u] = s0 + u < a.splits ? a.outp[((int64_t)(s0 + u) * a.n + i) * R + c] : 0.0;
#pragma unroll
        for (int u = 0; u < 8; ++u)
          if (s0 + u < a.splits) ky += t[u];
      }
      const double yic = (double)a.Y[i * a.ldy + c];
      ky += alpha * yic;
      const double v = ky + (sigma2 + (a.col_shift ? a.col_shift[c] : 0.0)) * yic;
      if (a.out) a.out[i * a.ldo + c] = (float)v;
      if (a.D) {
        const double dic = (double)a.D[i * a.ldd + c];
        q = dic * v;
        if (has_grad) {
          const double wc = a.w ? a.w[c] : 1.0;
          gA += wc * dic * ky;
          gS += wc * (double)a.P[i * a.ldp + c] * (double)a.Q[i * a.ldq + c];
        }
      }
    }
    const double tt = bsum(q);
    if (threadIdx.x == 0) rec[a.nth + c] = tt;
  }
  const double tA = bsum(gA);
  const double tS = bsum(gS * sigma2);
  if (threadIdx.x == 0) {
    rec[0] = tA;
    for (int k = 1; k <= a.L; ++k) rec[k] = 0.0;
    rec[a.L + 1] = tS;
  }
}

template <int DPX, int RP, int GM>
static void stage_xm(const XArgs &xa, hipStream_t s) {
  const int64_t ntl = (xa.n + TJ - 1) / TJ;
  const int64_t nch = ntl * (XTile<DPX, RP, GM>::kBytes / 16);
  stage_tiles_xm<DPX, RP, GM><<<(unsigned)((nch + 255) / 256), 256, 0, s>>>(xa, ntl);
}

template <int DPX, int RP>
static void launch_dr(const XArgs &xa, int gm, dim3 grid, hipStream_t s) {
  if (gm == 0) {
    stage_xm<DPX, RP, 0>(xa, s);
    pair_xm<DPX, RP, 0, 2><<<grid, kWG, 0, s>>>(xa);
  } else if (gm == 1) {
    stage_xm<DPX, RP, 1>(xa, s);
    pair_xm<DPX, RP, 1, 2><<<grid, kWG, 0, s>>>(xa);
  } else {
    stage_xm<DPX, RP, 2>(xa, s);
    pair_xm<DPX, RP, 2, 1><<<grid, kWG, 0, s>>>(xa);
  }
}

}  // namespace xm

int xm_rows_per_block(int has_grad_ard) { return xm::kWaves * 16 * (has_grad_ard ? 1 : 2); }
int xm_dpx(int d) { return d <= 32 ? 32 : 64; }
// staged tiles sized for the largest layout of the width: R = 32 with the per-coordinate gradient
static size_t xm_stage_bytes(int64_t n, int dpx) {
  const size_t tile = dpx == 32 ? xm::XTile<32, 32, 2>::kBytes : xm::XTile<64, 32, 2>::kBytes;
  return align256((size_t)((n + xm::TJ - 1) / xm::TJ) * tile);
}
size_t xm_scratch_bytes(int64_t n, int d) {
  const int dpx = xm_dpx(d);
  return align256(sizeof(float) * 3 * xm::kAmaxBlocks + 64) + 2 * align256(2 * (size_t)n * dpx) +
         align256(4 * (size_t)n) + xm_stage_bytes(n, dpx);
}

hipError_t launch_pass_xm(const PassDesc &p, hipStream_t s) {
  using namespace xm;
  const int dpx = xm_dpx(p.d);
  char *scr = (char *)p.mfma_scratch;
  float *amax = (float *)scr;
  int *scl = (int *)(scr + sizeof(float) * 3 * kAmaxBlocks);
  char *o = scr + align256(sizeof(float) * 3 * kAmaxBlocks + 64);
  uint16_t *xh = (uint16_t *)o;
  o += align256(2 * (size_t)p.n * dpx);
  uint16_t *xl = (uint16_t *)o;
  o += align256(2 * (size_t)p.n * dpx);
  float *nrm = (float *)o;
  o += align256(4 * (size_t)p.n);
  u32x4 *stage = (u32x4 *)o;

  XArgs a;
  a.n = p.n;
  a.R = p.R;
  a.L = p.kind == 0 ? 1 : p.d;
  a.d = p.d;
  a.xs = (const float *)p.xs;
  a.xst = p.dp;
  a.xh = xh;
  a.xl = xl;
  a.nrm = nrm;
  a.theta = p.theta;
  a.Y = (const float *)p.Y;
  a.ldy = p.ldy;
  a.P = (const float *)p.P;
  a.ldp = p.ldp;
  a.Q = (const float *)p.Q;
  a.ldq = p.ldq;
  a.w = p.w;
  a.D = (const float *)p.D;
  a.ldd = p.ldd;
  a.col_shift = p.col_shift;
  a.no_noise = p.no_noise;
  a.out = (float *)p.out;
  a.ldo = p.ldo;
  a.splits = p.splits;
  // column chunks of the split grid are whole tiles, so no tile straddles two splits
  a.col_chunk = ((p.n + p.splits - 1) / p.splits + TJ - 1) / TJ * TJ;
  a.outp = p.outp;
  a.rec = p.rec_pair;
  a.nth = p.nth;
  a.nrec = p.nrec;
  a.scl = scl;
  a.amax = amax;
  a.stage = stage;
  const int gm = p.P ? (p.kind == 0 ? 1 : 2) : 0;
  xm_prep<<<(unsigned)((p.n + 255) / 256), 256, 0, s>>>((const float *)p.xs, p.n, p.dp, dpx, xh,
                                                       xl, nrm);
  absmax_partial<<<dim3(kAmaxBlocks, 3), 256, 0, s>>>(a);
  scales_final<<<1, 64, 0, s>>>(a, scl);
  const int rp = p.R <= 16 ? 16 : 32;
  const int rows = xm_rows_per_block(gm == 2);
  dim3 grid((unsigned)((p.n + rows - 1) / rows), (unsigned)p.splits);
  if (dpx == 32) {
    if (rp == 16) launch_dr<32, 16>(a, gm, grid, s); else launch_dr<32, 32>(a, gm, grid, s);
  } else {
    if (rp == 16) launch_dr<64, 16>(a, gm, grid, s); else launch_dr<64, 32>(a, gm, grid, s);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (p.splits > 1) {
    XArgs f = a;
    f.rec = p.rec_fin;
    finalise_xm<<<(unsigned)((p.n + 255) / 256), 256, 0, s>>>(f, gm ? 1 : 0);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace gpk
