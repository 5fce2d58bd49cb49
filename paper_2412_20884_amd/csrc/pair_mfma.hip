// Matrix-core pair kernel for float inputs: the two R-wide contractions of every pair tile run on
// gfx950 MFMA (v_mfma_f32_16x16x32_f16) with operands split into float16 hi + lo parts, three
// products per contraction (hi*hi + hi*lo + lo*hi) and float accumulation; distances, exp2,
// splits and gradient sums run on the VALU.
//
// Per pair tile (32 columns j x 16 rows i per MFMA block):
//   S^T[j][i] = sum_c Q_jc (w_c P_ic)             (quad weights; MFMA, k = c)
//   K[i][j]  = exp2(log2 alpha - rho_ij)           (VALU; rho from scaled direct differences)
//   W = K S, g_l += W rho (iso) or W (x~_ik - x~_jk)^2 (ARD)   (VALU)
//   out[i][c] += sum_j K[i][j] Y_jc                (MFMA, k = j)
// The 16x16x32 operand layouts (lane l = 16 g + m): A[m][8g + q], B[8g + q][m], D[4g + r][m].
// The D layout of S^T gives lane l the values K[i = m][j = 4g + r] of two 16-column halves of
// the tile, which are exactly the eight A-operand values of the K*Y product once its k index
// is ordered as slot 8g + q <-> j = 16 (q / 4) + 4 g + (q % 4); the transposed Y tile in LDS
// is stored in that slot order.
//
// Range: every split operand is scaled by a power of two so its largest magnitude is below
// 2^14 (kernel values through the exp2 argument, Y, P*w and Q through a max reduction); the
// scales are removed when the float partial sums are folded into double accumulators.
//
// The sum of W over pairs (the log alpha gradient) is not accumulated per pair: it equals
// sum_ic w_c D_ic (K Y)_ic and is formed from the row results (D is the operand paired with Y).
//
// Column side: a pre-pass (stage_tiles) writes every 64-column tile once per call, split,
// scaled and laid out byte for byte as the LDS tile; the pair kernel streams the next tile into
// its second LDS buffer with direct global-to-LDS copies while it computes the current one.
#include "pass.h"

namespace gpk {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef __fp16 f16x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

namespace mf {

constexpr int kWaves = 8;
constexpr int kWG = kWaves * 64;  // 512 threads
constexpr int TH = 32;            // columns per MFMA half-tile
constexpr int NHALF = 2;          // half-tiles per LDS tile (one barrier interval)
constexpr int TJ = TH * NHALF;    // columns per LDS tile
constexpr int kStrideH = 40;      // halves per LDS row of the split tiles (80 bytes)
constexpr int kFold = 4;          // tiles (of 64 columns) between folds of the float partials
constexpr int kScaleTop = 14;     // operands scaled below 2^14
constexpr int kAmaxBlocks = 64;

// A column tile as stage_tiles lays it out in global memory, byte for byte the image of one
// LDS tile buffer: Y^T hi and Y^T lo (a padded row of 32 slot-ordered halves per (half, column
// c)), then with the gradient Q hi and Q lo (a padded row of 32 halves per point, c >= RP zero),
// then the coordinates (XS floats per point), rounded up to whole 1 KB wave copies.
template <int RP, int XS, int GM>
struct TileGeom {
  static constexpr int kRowB = kStrideH * 2;
  static constexpr int kYB = NHALF * RP * kRowB;
  static constexpr int kQB = GM ? TJ * kRowB : 0;
  static constexpr int kXB = TJ * XS * 4;
  static constexpr int kOffYL = kYB;
  static constexpr int kOffQH = 2 * kYB;
  static constexpr int kOffQL = 2 * kYB + kQB;
  static constexpr int kOffX = 2 * kYB + 2 * kQB;
  static constexpr int kBytes = (kOffX + kXB + 1023) / 1024 * 1024;
};

union H8 {
  f16x8 v;
  uint32_t u[4];
};

__device__ __forceinline__ uint32_t pk_rtz(float a, float b) {
  f16x2 h = __builtin_amdgcn_cvt_pkrtz(a, b);
  return __builtin_bit_cast(uint32_t, h);
}

// Split a float into hi (10 explicit mantissa bits, exact in float16 in the normal range) and lo.
__device__ __forceinline__ void split(float x, float &hi, float &lo) {
  hi = __uint_as_float(__float_as_uint(x) & 0xFFFFE000u);
  lo = x - hi;
}

struct MArgs {
  int64_t n;
  int R;
  int L;
  const float *xs;  // n x 4|8|16 scaled coordinates
  int xstride;
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
  const int *scl;  // [0] eK (from theta), [1] eY, [2] eP, [3] eQ
  float *amax;     // [3][kAmaxBlocks] partial max |.| of Y, P*w, Q
  u32x4 *stage;    // column tiles laid out by stage_tiles
};

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  return v;
}

__global__ __launch_bounds__(256) void absmax_partial(MArgs a) {
  __shared__ float sh[4];
  const int which = blockIdx.y;  // 0 Y, 1 P*w, 2 Q
  const float *A = which == 0 ? a.Y : (which == 1 ? a.P : a.Q);
  const int64_t ld = which == 0 ? a.ldy : (which == 1 ? a.ldp : a.ldq);
  float m = 0.0f;
  if (A) {
    const int64_t ne = a.n * a.R;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < ne;
         e += (int64_t)gridDim.x * 256) {
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
  frexpf(m, &e);  // m < 2^e
  e = kScaleTop - e;
  return e > 100 ? 100 : (e < -100 ? -100 : e);
}

__global__ void scales_final(MArgs a, int *scl) {
  if (threadIdx.x != 0) return;
  // kernel values: alpha * 2^eK <= 2^14
  const double l2a = a.theta[0] * kLog2e;
  int eK = kScaleTop - (int)ceil(l2a);
  if (eK > 100) eK = 100;
  if (eK < -100) eK = -100;
  scl[0] = eK;
  for (int which = 0; which < 3; ++which) {
    float m = 0.0f;
    for (int b = 0; b < kAmaxBlocks; ++b) m = fmaxf(m, a.amax[which * kAmaxBlocks + b]);
    scl[1 + which] = scale_exp(m);
  }
}

// Split, scale and lay out the column side of every 64-column tile in the order of the pair
// kernel's LDS tile (TileGeom): Y^T hi and lo with column jl of half hh in slot 8 gg + q
// (gg = (jl mod 16) / 4, q = 4 (jl / 16) + jl mod 4), Q hi and lo, and the coordinates.
// Columns past n get Y = Q = 0 and a far-away point, so their kernel values vanish.
template <int RP, int XS, int GM>
__global__ __launch_bounds__(256) void stage_tiles(MArgs a, int64_t ntiles) {
  using G = TileGeom<RP, XS, GM>;
  constexpr int kCh = G::kBytes / 16;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= ntiles * kCh) return;
  const int64_t tile = e / kCh;
  const int off = 16 * (int)(e - tile * kCh);
  const int64_t jt = tile * TJ;
  union {
    u32x4 v;
    _Float16 h[8];
    float f[4];
  } out;
  out.v = u32x4{0u, 0u, 0u, 0u};
  if (off < G::kOffQH) {
    const bool lo = off >= G::kOffYL;
    const int o = off - (lo ? G::kOffYL : 0);
    const int row = o / G::kRowB, cb = o - row * G::kRowB;  // row = hh RP + c
    if (cb < 64) {
      const float sY = ldexpf(1.0f, a.scl[1]);
      const int q = cb >> 4;  // slots 8 q .. 8 q + 7
      const int hh = row / RP, c = row - hh * RP;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int jl = 16 * (u >> 2) + 4 * q + (u & 3);
        const int64_t j = jt + 32 * hh + jl;
        float h, l;
        split((j < a.n && c < a.R) ? a.Y[j * a.ldy + c] * sY : 0.0f, h, l);
        out.h[u] = (_Float16)(lo ? l : h);
      }
    }
  } else if (off < G::kOffX) {
    const bool lo = off >= G::kOffQL;
    const int o = off - (lo ? G::kOffQL : G::kOffQH);
    const int jj = o / G::kRowB, cb = o - jj * G::kRowB;
    if (cb < 2 * RP) {
      const float sQ = ldexpf(1.0f, a.scl[3]);
      const int64_t j = jt + jj;
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int c = cb / 2 + u;
        float h, l;
        split((j < a.n && c < a.R) ? a.Q[j * a.ldq + c] * sQ : 0.0f, h, l);
        out.h[u] = (_Float16)(lo ? l : h);
      }
    }
  } else if (off < G::kOffX + G::kXB) {
    const int f0 = (off - G::kOffX) / 4;
    const int jj = f0 / XS, k0 = f0 - jj * XS;
    const int64_t j = jt + jj;
#pragma unroll
    for (int u = 0; u < 4; ++u)
      out.f[u] = j < a.n ? a.xs[j * XS + k0 + u] : (k0 + u == 0 ? 1.0e18f : 0.0f);
  }
  a.stage[e] = out.v;
}

// GM: 0 product only, 1 isotropic gradient, 2 per-coordinate gradient.
// D: coordinates used (1..4 stored with stride 4, or 8, 16).  RP: padded R (16 or 32).
// IB: 16-row blocks per wave (1 or 2; the per-coordinate gradient at d >= 8 always uses 1,
// its accumulators need the registers of the second block).
template <int D, int RP, int GM, int IB>
__global__ __launch_bounds__(kWG) void pair_mfma(MArgs a) {
  constexpr int kRowsWG = kWaves * IB * 16;
  constexpr int XS = D <= 4 ? 4 : D;         // LDS/global stride of a point
  constexpr int NCB = RP / 16;               // 16-column blocks of the product
  constexpr int NG = GM == 2 ? D : 1;
  // LDS: double-buffered tile
  using G = TileGeom<RP, XS, GM>;
  __shared__ __attribute__((aligned(16))) char tile0[G::kBytes];
  __shared__ __attribute__((aligned(16))) char tile1[G::kBytes];
  __shared__ double shr[kWaves][4];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int m = lane & 15, g = lane >> 4;
  const int64_t row0 = (int64_t)blockIdx.x * kRowsWG + wave * (IB * 16);
  const int R = a.R;

  const int eK = a.scl[0], eY = a.scl[1], eP = a.scl[2], eQ = a.scl[3];
  const float c0 = (float)(a.theta[0] * kLog2e + (double)eK);

  // ---- row side: coordinates and the split weighted P operand (B of the S^T product) ----
  float xi[IB][D];
  H8 ph[IB], pl[IB];
#pragma unroll
  for (int ib = 0; ib < IB; ++ib) {
    int64_t i = row0 + ib * 16 + m;
    // rows past the end reuse the last row's coordinates but get a zero P operand, so their
    // quad weights, and with them every gradient contribution, vanish
    const bool row_ok = i < a.n;
    if (!row_ok) i = a.n - 1;
#pragma unroll
    for (int k = 0; k < D; ++k) xi[ib][k] = a.xs[i * XS + k];
    if (GM) {
      const float sP = ldexpf(1.0f, eP);
      float v[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int c = 8 * g + q;
        v[q] = (row_ok && c < R)
                   ? (float)((double)a.P[i * a.ldp + c] * (a.w ? a.w[c] : 1.0)) * sP
                   : 0.0f;
      }
#pragma unroll
      for (int q = 0; q < 8; q += 2) {
        float h0, l0, h1, l1;
        split(v[q], h0, l0);
        split(v[q + 1], h1, l1);
        ph[ib].u[q / 2] = pk_rtz(h0, h1);
        pl[ib].u[q / 2] = pk_rtz(l0, l1);
      }
    }
  }

  f32x4 acc[IB][NCB];
  double acc64[IB][NCB][4];
  // gradient partials: float per lane over kFold tiles, then (iso) a double per lane or
  // (ARD) a wave reduction into per-wave double slots in LDS
  float gl[NG];
  double gl64 = 0.0;
  __shared__ double glsh[kWaves][GM == 2 ? D : 1];
#pragma unroll
  for (int ib = 0; ib < IB; ++ib)
#pragma unroll
    for (int cb = 0; cb < NCB; ++cb) {
      acc[ib][cb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int r = 0; r < 4; ++r) acc64[ib][cb][r] = 0.0;
    }
#pragma unroll
  for (int k = 0; k < NG; ++k) gl[k] = 0.0f;
  if (GM == 2 && lane < NG) glsh[wave][lane] = 0.0;
  const double unscale_out = ldexp(1.0, -(eK + eY));
  const double unscale_g = ldexp(1.0, -(eK + eP + eQ));

  const int64_t j0 = (int64_t)blockIdx.y * a.col_chunk;
  const int64_t j1 = j0 + a.col_chunk < a.n ? j0 + a.col_chunk : a.n;
  const int ntiles = (int)((j1 - j0 + TJ - 1) / TJ);
  // Column tiles (64 columns = two 32-column MFMA halves) are double-buffered: while tile t is
  // computed from one LDS buffer, tile t + 1 streams into the other by direct global-to-LDS
  // copies (each wave moves whole 1 KB blocks of the tile image stage_tiles wrote), and every
  // wave waits for its copies before the barrier that ends the tile.
  constexpr int kRounds = (G::kBytes / 1024 + kWaves - 1) / kWaves;
  const char *gtiles = (const char *)a.stage + (j0 / TJ) * (int64_t)G::kBytes + lane * 16;
  auto issue = [&](int t, char *dst) {
    const char *src = gtiles + (int64_t)t * G::kBytes;
#pragma unroll
    for (int u = 0; u < kRounds; ++u) {
      const int off = (u * kWaves + wave) * 1024;
      if (off < G::kBytes)
        __builtin_amdgcn_global_load_lds(src + off,
                                         (__attribute__((address_space(3))) void *)(dst + off),
                                         16, 0, 0);
    }
  };
  if (ntiles > 0) issue(0, tile0);
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  // two steps per loop trip, so that every LDS access names its buffer statically and the
  // copies into one buffer do not hold up the reads of the other
  auto tile_step = [&](int t, const char *cur, char *nxt) {
    if (t + 1 < ntiles) issue(t + 1, nxt);
    // both halves unrolled (constant LDS offsets) except for the per-coordinate gradient,
    // whose accumulators leave no registers for it
    constexpr int kHalfUnroll = GM == 2 ? 1 : NHALF;
#pragma unroll kHalfUnroll
    for (int hf = 0; hf < NHALF; ++hf) {
      // ---- S^T for both 16-column quarters of this half and all row blocks ---------------
      f32x4 s[IB][2];
      if (GM) {
#pragma unroll
        for (int jb = 0; jb < 2; ++jb) {
          H8 vh, vl;
          const int row = 32 * hf + 16 * jb + m;
          vh.v = *(const f16x8 *)(cur + G::kOffQH + 2 * (row * kStrideH + 8 * g));
          vl.v = *(const f16x8 *)(cur + G::kOffQL + 2 * (row * kStrideH + 8 * g));
#pragma unroll
          for (int ib = 0; ib < IB; ++ib) {
            f32x4 z = {0.f, 0.f, 0.f, 0.f};
            z = __builtin_amdgcn_mfma_f32_16x16x32_f16(vh.v, ph[ib].v, z, 0, 0, 0);
            z = __builtin_amdgcn_mfma_f32_16x16x32_f16(vh.v, pl[ib].v, z, 0, 0, 0);
            z = __builtin_amdgcn_mfma_f32_16x16x32_f16(vl.v, ph[ib].v, z, 0, 0, 0);
            s[ib][jb] = z;
          }
        }
      }
      // ---- kernel values (VALU) into the A operand of the product -------------------------
      H8 kh[IB], kl[IB];
#pragma unroll
      for (int jb = 0; jb < 2; ++jb) {
        float kv[IB][4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          float xj[D];
          const float *p0 = (const float *)(cur + G::kOffX) + (32 * hf + 16 * jb + 4 * g + r) * XS;
#pragma unroll
          for (int k = 0; k < D; ++k) xj[k] = p0[k];
#pragma unroll
          for (int ib = 0; ib < IB; ++ib) {
            // the product-only pass takes the exp2 argument c0 - rho straight from the FMA
            // chain; the gradient passes need rho itself (folding c0 there would cancel
            // badly against the rho = 0 diagonal pairs in sum W rho)
            float d2[GM == 2 ? D : 1];
            float rho = 0.f, arg = c0;
#pragma unroll
            for (int k = 0; k < D; ++k) {
              const float u = xi[ib][k] - xj[k];
              if (GM == 2) {
                d2[k] = u * u;
                rho += d2[k];
              } else if (GM == 1) {
                rho = fmaf(u, u, rho);
              } else {
                arg = fmaf(-u, u, arg);
              }
            }
            const float kk = __builtin_amdgcn_exp2f(GM ? c0 - rho : arg);
            if (GM) {
              const float W = kk * s[ib][jb][r];
              if (GM == 1) {
                gl[0] = fmaf(W, rho, gl[0]);
              } else {
#pragma unroll
                for (int k = 0; k < D; ++k) gl[k] = fmaf(W, d2[k], gl[k]);
              }
            }
            kv[ib][r] = kk;
          }
        }
#pragma unroll
        for (int ib = 0; ib < IB; ++ib) {
#pragma unroll
          for (int r = 0; r < 4; r += 2) {
            float h0, l0, h1, l1;
            split(kv[ib][r], h0, l0);
            split(kv[ib][r + 1], h1, l1);
            kh[ib].u[2 * jb + r / 2] = pk_rtz(h0, h1);
            kl[ib].u[2 * jb + r / 2] = pk_rtz(l0, l1);
          }
        }
      }
      // ---- product out += K Y -------------------------------------------------------------
#pragma unroll
      for (int cb = 0; cb < NCB; ++cb) {
        H8 yh, yl;
        yh.v = *(const f16x8 *)(cur + 2 * ((hf * RP + 16 * cb + m) * kStrideH + 8 * g));
        yl.v = *(const f16x8 *)(cur + G::kOffYL + 2 * ((hf * RP + 16 * cb + m) * kStrideH + 8 * g));
#pragma unroll
        for (int ib = 0; ib < IB; ++ib) {
          f32x4 z = acc[ib][cb];
          z = __builtin_amdgcn_mfma_f32_16x16x32_f16(kh[ib].v, yh.v, z, 0, 0, 0);
          z = __builtin_amdgcn_mfma_f32_16x16x32_f16(kh[ib].v, yl.v, z, 0, 0, 0);
          z = __builtin_amdgcn_mfma_f32_16x16x32_f16(kl[ib].v, yh.v, z, 0, 0, 0);
          acc[ib][cb] = z;
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
        gl64 += (double)gl[0];
        gl[0] = 0.0f;
      } else if (GM == 2) {
#pragma unroll
        for (int k = 0; k < NG; ++k) {
          const double v = wave_sum((double)gl[k]);
          if (lane == 0) glsh[wave][k] += v;
          gl[k] = 0.0f;
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
  // Lane holds (K Y)[i = row0 + 16 ib + 4 g + r][c = 16 cb + m] (scaled).
  const int64_t blk = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
  double *rec = a.rec + blk * a.nrec;
  const double sigma2 = a.no_noise ? 0.0 : exp(a.theta[a.nth - 1]);
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
          const double ky = acc64[ib][cb][r] * unscale_out;
          if (a.splits == 1) {
            const double yic = (double)a.Y[i * a.ldy + c];
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
            a.outp[((int64_t)blockIdx.y * a.n + i) * R + c] = ky;
          }
        }
      }
    }
  gS *= sigma2;
  // record: block reductions (lanes sharing a column c = 16 cb + m sum over g and waves)
  __shared__ double sred[kWaves][64];
  auto block_total = [&](double v) -> double {
    v = wave_sum(v);
    __syncthreads();
    if (lane == 0) shr[wave][0] = v;
    __syncthreads();
    double t = 0.0;
    for (int w_ = 0; w_ < kWaves; ++w_) t += shr[w_][0];
    return t;
  };
  {
    const double t = block_total(gA);
    if (tid == 0) rec[0] = t;
  }
  for (int k = 0; k < a.L; ++k) {
    double t;
    if (GM == 2) {
      __syncthreads();
      t = 0.0;
      for (int w_ = 0; w_ < kWaves; ++w_) t += glsh[w_][k];
      t *= unscale_g;
    } else {
      t = block_total(GM == 1 ? gl64 * unscale_g : 0.0);
    }
    if (tid == 0) rec[1 + k] = t;
  }
  {
    const double t = block_total(gS);
    if (tid == 0) rec[a.L + 1] = t;
  }
  // per-column quad sums: lanes m, m+16, m+32, m+48 of every wave hold column 16 cb + m
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
      double t = 0.0;
      for (int w_ = 0; w_ < kWaves; ++w_) t += sred[w_][tid];
      if (c < R) rec[a.nth + c] = t;
    }
  }
}

// Column-split partials: sum the splits of (K Y), add the diagonal, write the output and the
// records of q_c, the log alpha gradient (sum_ic w_c D_ic (K Y)_ic) and the sigma^2 term.
__global__ __launch_bounds__(256) void finalise_mfma(MArgs a, int has_grad) {
  __shared__ double sh4[4];
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool live = i < a.n;
  const int R = a.R;
  const double sigma2 = a.no_noise ? 0.0 : exp(a.theta[a.nth - 1]);
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
    const double t = bsum(q);
    if (threadIdx.x == 0) rec[a.nth + c] = t;
  }
  const double tA = bsum(gA);
  const double tS = bsum(gS * sigma2);
  if (threadIdx.x == 0) {
    rec[0] = tA;
    for (int k = 1; k <= a.L; ++k) rec[k] = 0.0;
    rec[a.L + 1] = tS;
  }
}

template <int D, int RP, int GM>
static void launch_d_rp_gm(const MArgs &ma, int ib, dim3 grid, hipStream_t s) {
  constexpr int XS = D <= 4 ? 4 : D;
  const int64_t ntl = (ma.n + TJ - 1) / TJ;
  const int64_t nch = ntl * (TileGeom<RP, XS, GM>::kBytes / 16);
  stage_tiles<RP, XS, GM><<<(unsigned)((nch + 255) / 256), 256, 0, s>>>(ma, ntl);
  if constexpr (GM == 2 && D >= 8) {
    pair_mfma<D, RP, GM, 1><<<grid, kWG, 0, s>>>(ma);
  } else {
    if (ib == 1)
      pair_mfma<D, RP, GM, 1><<<grid, kWG, 0, s>>>(ma);
    else
      pair_mfma<D, RP, GM, 2><<<grid, kWG, 0, s>>>(ma);
  }
}

template <int D, int RP>
static void launch_d_rp(const MArgs &ma, int gm, int ib, dim3 grid, hipStream_t s) {
  if (gm == 0)
    launch_d_rp_gm<D, RP, 0>(ma, ib, grid, s);
  else if (gm == 1)
    launch_d_rp_gm<D, RP, 1>(ma, ib, grid, s);
  else
    launch_d_rp_gm<D, RP, 2>(ma, ib, grid, s);
}

}  // namespace mf

int mfma_ib(int kind, int d, int has_grad, int ib_request) {
  if (has_grad && kind != 0 && d > 4) return 1;
  return ib_request == 1 ? 1 : 2;
}

int mfma_rows_per_block(int kind, int d, int has_grad, int ib_request) {
  return mf::kWaves * 16 * mfma_ib(kind, d, has_grad, ib_request);
}

namespace mf {

template <int D>
static void launch_d(const MArgs &ma, int rp, int gm, int ib, dim3 grid, hipStream_t s) {
  if (rp == 16)
    launch_d_rp<D, 16>(ma, gm, ib, grid, s);
  else
    launch_d_rp<D, 32>(ma, gm, ib, grid, s);
}

}  // namespace mf

bool mfma_supported(int prec, int kind, int d, int R) {
  (void)kind;
  return prec == kF32 && d <= 16 && R >= 8 && R <= 32;
}

static size_t mfma_head_bytes() { return align256(sizeof(float) * 3 * mf::kAmaxBlocks + 64); }

// Extra workspace of the matrix-core pass: partial maxima, the four scale exponents and the
// staged column tiles (sized for R = 32 with the gradient operand).
size_t mfma_scratch_bytes(int64_t n, int dp) {
  const int64_t ntl = (n + mf::TJ - 1) / mf::TJ;
  const size_t tile = ((size_t)4 * mf::TJ * mf::kStrideH * 2 + (size_t)mf::TJ * dp * 4 + 1023) /
                      1024 * 1024;
  return mfma_head_bytes() + align256((size_t)ntl * tile);
}

hipError_t launch_pass_mfma(const PassDesc &p, hipStream_t s) {
  using namespace mf;
  MArgs a;
  a.n = p.n;
  a.R = p.R;
  a.L = p.kind == 0 ? 1 : p.d;
  a.xs = (const float *)p.xs;
  a.xstride = p.dp;
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
  a.amax = (float *)p.mfma_scratch;
  int *scl = (int *)((char *)p.mfma_scratch + sizeof(float) * 3 * kAmaxBlocks);
  a.scl = scl;
  a.stage = (u32x4 *)((char *)p.mfma_scratch + mfma_head_bytes());
  const int gm = p.P ? (p.kind == 0 ? 1 : 2) : 0;
  absmax_partial<<<dim3(kAmaxBlocks, 3), 256, 0, s>>>(a);
  scales_final<<<1, 64, 0, s>>>(a, scl);
  const int rp = p.R <= 16 ? 16 : 32;
  const int ib = mfma_ib(p.kind, p.d, gm ? 1 : 0, p.ib);
  const int rows = mfma_rows_per_block(p.kind, p.d, gm ? 1 : 0, p.ib);
  dim3 grid((unsigned)((p.n + rows - 1) / rows), (unsigned)p.splits);
  const int dd = p.d;
  if (dd == 1)
    launch_d<1>(a, rp, gm, ib, grid, s);
  else if (dd == 2)
    launch_d<2>(a, rp, gm, ib, grid, s);
  else if (dd == 3)
    launch_d<3>(a, rp, gm, ib, grid, s);
  else if (dd == 4)
    launch_d<4>(a, rp, gm, ib, grid, s);
  else if (dd <= 8)
    launch_d<8>(a, rp, gm, ib, grid, s);
  else
    launch_d<16>(a, rp, gm, ib, grid, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (p.splits > 1) {
    MArgs f = a;
    f.rec = p.rec_fin;
    finalise_mfma<<<(unsigned)((p.n + 255) / 256), 256, 0, s>>>(f, gm ? 1 : 0);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace gpk
