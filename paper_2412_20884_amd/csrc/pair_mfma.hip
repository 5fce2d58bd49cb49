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

// A column tile as stage_tiles lays it out in global memory: 16-byte chunks of Y^T hi, Y^T lo
// (one row of 32 slot-ordered halves per (half, column c)), then with the gradient Q hi and Q lo
// (one row of RP halves per point), then the coordinates (XS floats per point).
template <int RP, int XS, int GM>
struct StageGeom {
  static constexpr int kYC = NHALF * RP * 4;
  static constexpr int kQC = GM ? TJ * RP / 8 : 0;
  static constexpr int kXC = TJ * XS / 4;
  static constexpr int kChunks = 2 * kYC + 2 * kQC + kXC;
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
// kernel's LDS tile (StageGeom): Y^T hi and lo with column jl of half hh in slot 8 gg + q
// (gg = (jl mod 16) / 4, q = 4 (jl / 16) + jl mod 4), Q hi and lo, and the coordinates.
// Columns past n get Y = Q = 0 and a far-away point, so their kernel values vanish.
template <int RP, int XS, int GM>
__global__ __launch_bounds__(256) void stage_tiles(MArgs a, int64_t ntiles) {
  using G = StageGeom<RP, XS, GM>;
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= ntiles * G::kChunks) return;
  const int64_t tile = e / G::kChunks;
  int k = (int)(e - tile * G::kChunks);
  const int64_t jt = tile * TJ;
  union {
    u32x4 v;
    _Float16 h[8];
    float f[4];
  } out;
  if (k < 2 * G::kYC) {
    const bool lo = k >= G::kYC;
    if (lo) k -= G::kYC;
    const float sY = ldexpf(1.0f, a.scl[1]);
    const int row = k >> 2, q = k & 3;  // row = hh RP + c; slots 8 q .. 8 q + 7
    const int hh = row / RP, c = row - hh * RP;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int jl = 16 * (u >> 2) + 4 * q + (u & 3);
      const int64_t j = jt + 32 * hh + jl;
      float h, l;
      split((j < a.n && c < a.R) ? a.Y[j * a.ldy + c] * sY : 0.0f, h, l);
      out.h[u] = (_Float16)(lo ? l : h);
    }
  } else if (GM && k < 2 * G::kYC + 2 * G::kQC) {
    k -= 2 * G::kYC;
    const bool lo = k >= G::kQC;
    if (lo) k -= G::kQC;
    const float sQ = ldexpf(1.0f, a.scl[3]);
    constexpr int kPerRow = RP / 8;
    const int jj = k / kPerRow, c0 = 8 * (k - jj * kPerRow);
    const int64_t j = jt + jj;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int c = c0 + u;
      float h, l;
      split((j < a.n && c < a.R) ? a.Q[j * a.ldq + c] * sQ : 0.0f, h, l);
      out.h[u] = (_Float16)(lo ? l : h);
    }
  } else {
    k -= 2 * G::kYC + 2 * G::kQC;
    const int jj = (4 * k) / XS, k0 = 4 * k - jj * XS;
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
  __shared__ __attribute__((aligned(16))) float sx[2][TJ * XS];
  __shared__ __attribute__((aligned(16))) _Float16 sqh[2][TJ * kStrideH];   // Q[j][c]
  __shared__ __attribute__((aligned(16))) _Float16 sql[2][TJ * kStrideH];
  __shared__ __attribute__((aligned(16))) _Float16 syh[2][NHALF * RP * kStrideH];  // Y^T[h][c][slot]
  __shared__ __attribute__((aligned(16))) _Float16 syl[2][NHALF * RP * kStrideH];
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
  // Column tiles (64 columns = two 32-column MFMA halves) are software-pipelined: tile t + 2 is
  // loaded into registers after the compute of tile t, and tile t + 1 is written to the other
  // LDS buffer.  Tiles arrive split and ordered from stage_tiles; every thread copies the same
  // 16-byte chunk positions of every tile, so the destinations are fixed per thread.
  using G = StageGeom<RP, XS, GM>;
  constexpr int NCT = (G::kChunks + kWG - 1) / kWG;  // chunks per thread per tile
  const u32x4 *stile = a.stage + (j0 / TJ) * G::kChunks;
  u32x4 rv[NCT];
  int dreg[NCT], doff[NCT];  // LDS region (0 Y hi, 1 Y lo, 2 Q hi, 3 Q lo, 4 coordinates), offset
#pragma unroll
  for (int u = 0; u < NCT; ++u) {
    int k = tid + u * kWG;
    if (k < 2 * G::kYC) {
      dreg[u] = k >= G::kYC;
      k -= dreg[u] * G::kYC;
      doff[u] = (k >> 2) * kStrideH + 8 * (k & 3);
    } else if (k < 2 * G::kYC + 2 * G::kQC) {
      k -= 2 * G::kYC;
      const int lo = k >= G::kQC;
      dreg[u] = 2 + lo;
      k -= lo * G::kQC;
      constexpr int kPerRow = RP / 8;
      doff[u] = (k / kPerRow) * kStrideH + 8 * (k % kPerRow);
    } else {
      dreg[u] = 4;
      doff[u] = 4 * (k - 2 * G::kYC - 2 * G::kQC);
    }
  }
  auto prefetch = [&](int t) {
    const u32x4 *src = stile + (int64_t)t * G::kChunks;
#pragma unroll
    for (int u = 0; u < NCT; ++u)
      if (tid + u * kWG < G::kChunks) rv[u] = src[tid + u * kWG];
  };
  auto commit = [&](int b) {
#pragma unroll
    for (int u = 0; u < NCT; ++u) {
      if (tid + u * kWG < G::kChunks) {
        switch (dreg[u]) {  // uniform per wave: region sizes are multiples of 64 chunks
          case 0: *(u32x4 *)&syh[b][doff[u]] = rv[u]; break;
          case 1: *(u32x4 *)&syl[b][doff[u]] = rv[u]; break;
          case 2: *(u32x4 *)&sqh[b][doff[u]] = rv[u]; break;
          case 3: *(u32x4 *)&sql[b][doff[u]] = rv[u]; break;
          default: *(u32x4 *)&sx[b][doff[u]] = rv[u]; break;
        }
      }
    }
  };
  if (GM && RP < 32) {
    // the unused half of the S contraction (c = RP .. 31) stays zero in both buffers
    for (int e = tid; e < 2 * TJ * (32 - RP); e += kWG) {
      const int bb = e / (TJ * (32 - RP));
      const int r2 = e - bb * TJ * (32 - RP);
      const int jj = r2 / (32 - RP), c = RP + (r2 - jj * (32 - RP));
      sqh[bb][jj * kStrideH + c] = (_Float16)0.0f;
      sql[bb][jj * kStrideH + c] = (_Float16)0.0f;
    }
  }

  if (ntiles > 0) {
    prefetch(0);
    commit(0);
  }
  if (ntiles > 1) prefetch(1);
  __syncthreads();
  for (int t = 0; t < ntiles; ++t) {
    const int b = t & 1;
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
          vh.v = *(const f16x8 *)&sqh[b][row * kStrideH + 8 * g];
          vl.v = *(const f16x8 *)&sql[b][row * kStrideH + 8 * g];
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
          const float *p0 = &sx[b][(32 * hf + 16 * jb + 4 * g + r) * XS];
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
        yh.v = *(const f16x8 *)&syh[b][(hf * RP + 16 * cb + m) * kStrideH + 8 * g];
        yl.v = *(const f16x8 *)&syl[b][(hf * RP + 16 * cb + m) * kStrideH + 8 * g];
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
    if (t + 1 < ntiles) commit(b ^ 1);
    if (t + 2 < ntiles) prefetch(t + 2);
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
    __syncthreads();
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
      for (int s = 0; s < a.splits; ++s) ky += a.outp[((int64_t)s * a.n + i) * R + c];
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
  const int64_t nch = ntl * StageGeom<RP, XS, GM>::kChunks;
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
  const size_t chunks = (size_t)2 * mf::NHALF * 32 * 4 + (size_t)2 * mf::TJ * 32 / 8 +
                        (size_t)mf::TJ * dp / 4;
  return mfma_head_bytes() + align256((size_t)ntl * chunks * 16);
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
