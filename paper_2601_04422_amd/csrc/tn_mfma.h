// Complex 64x64 tile products on CDNA matrix cores (float32 accumulation).
//
// Operands are complex float32 tiles in LDS:  Af[row][k] (64 rows x 16 k)
// and Bf[col][k] (64 columns x 16 k, i.e. B transposed), row stride TILE_LD.
// A workgroup of 4 wavefronts owns a 64x64 output; wavefront w owns the
// 32x32 quarter (rows 32*(w/2), columns 32*(w%2)) as 2x2 tiles of 16x16.
//
// Modes
//   MODE_F32   : v_mfma_f32_16x16x4f32, products of float32 operands.
//   MODE_BF16X3: each float32 operand x = x0 + x1 + x2 in bf16 pieces
//                (x0 = bf16(x), x1 = bf16(x - x0), x2 = bf16(x - x0 - x1));
//                products x0y0 + x0y1 + x1y0 on v_mfma_f32_16x16x16bf16_1k.
//   MODE_BF16X6: adds x1y1 + x0y2 + x2y0, about float32 accuracy.
// The split follows Henry, Tang & Heinecke, "Leveraging the bfloat16
// artificial intelligence datatype for higher-precision computations"
// (ARITH 2019).
#pragma once
#include <hip/hip_runtime.h>

namespace tn {

enum { MODE_F32 = 1, MODE_BF16X3 = 2, MODE_BF16X6 = 3 };

typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

constexpr int TILE_K = 16;
constexpr int TILE_LD = TILE_K + 1;  // float2 stride of one LDS operand row

__device__ __forceinline__ unsigned short f2bf(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);  // round to nearest even
  return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float bf2f(unsigned short h) {
  return __uint_as_float(((unsigned)h) << 16);
}

// Split 4 floats into 3 bf16 pieces each (piece p of value j -> out[p][j]).
__device__ __forceinline__ void split4(const float v[4], bf16x4_t out[3]) {
#pragma unroll
  for (int j = 0; j < 4; j++) {
    unsigned short p0 = f2bf(v[j]);
    float r = v[j] - bf2f(p0);
    unsigned short p1 = f2bf(r);
    r = r - bf2f(p1);
    unsigned short p2 = f2bf(r);
    out[0][j] = (short)p0;
    out[1][j] = (short)p1;
    out[2][j] = (short)p2;
  }
}

__device__ __forceinline__ f32x4_t mfma_bf16(bf16x4_t a, bf16x4_t b, f32x4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4_t mfma_f32(float a, float b, f32x4_t c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// acc{R,I}[ti][tj] += (Af * Bf^T) over one 16-wide k slice.
template <int MODE>
__device__ __forceinline__ void cmma_step(const float2 *Af, const float2 *Bf, int wave, int lane,
                                          f32x4_t accR[2][2], f32x4_t accI[2][2]) {
  const int wr = (wave >> 1) * 32, wc = (wave & 1) * 32;
  const int l16 = lane & 15, lg = lane >> 4;
  if constexpr (MODE == MODE_F32) {
#pragma unroll
    for (int kk = 0; kk < 4; kk++) {
      const int k = kk * 4 + lg;
      float ar[2], ai[2], br[2], bi[2];
#pragma unroll
      for (int t = 0; t < 2; t++) {
        float2 a = Af[(wr + t * 16 + l16) * TILE_LD + k];
        float2 b = Bf[(wc + t * 16 + l16) * TILE_LD + k];
        ar[t] = a.x;
        ai[t] = a.y;
        br[t] = b.x;
        bi[t] = b.y;
      }
#pragma unroll
      for (int ti = 0; ti < 2; ti++)
#pragma unroll
        for (int tj = 0; tj < 2; tj++) {
          accR[ti][tj] = mfma_f32(ar[ti], br[tj], accR[ti][tj]);
          accR[ti][tj] = mfma_f32(-ai[ti], bi[tj], accR[ti][tj]);
          accI[ti][tj] = mfma_f32(ar[ti], bi[tj], accI[ti][tj]);
          accI[ti][tj] = mfma_f32(ai[ti], br[tj], accI[ti][tj]);
        }
    }
  } else {
    const int k0 = lg * 4;
    bf16x4_t Ar[2][3], Ai[2][3], An[2][3], Br[2][3], Bi[2][3];
#pragma unroll
    for (int t = 0; t < 2; t++) {
      float vr[4], vi[4], vn[4];
      const float2 *pa = Af + (wr + t * 16 + l16) * TILE_LD + k0;
#pragma unroll
      for (int j = 0; j < 4; j++) {
        vr[j] = pa[j].x;
        vi[j] = pa[j].y;
        vn[j] = -pa[j].y;
      }
      split4(vr, Ar[t]);
      split4(vi, Ai[t]);
      split4(vn, An[t]);
      const float2 *pb = Bf + (wc + t * 16 + l16) * TILE_LD + k0;
#pragma unroll
      for (int j = 0; j < 4; j++) {
        vr[j] = pb[j].x;
        vi[j] = pb[j].y;
      }
      split4(vr, Br[t]);
      split4(vi, Bi[t]);
    }
    // piece pairs, small terms first
    constexpr int NP = MODE == MODE_BF16X6 ? 6 : 3;
    constexpr int PA[6] = {2, 0, 1, 1, 0, 0};
    constexpr int PB[6] = {0, 2, 1, 0, 1, 0};
    constexpr int OFF = MODE == MODE_BF16X6 ? 0 : 3;
#pragma unroll
    for (int ti = 0; ti < 2; ti++)
#pragma unroll
      for (int tj = 0; tj < 2; tj++)
#pragma unroll
        for (int q = OFF; q < OFF + NP && q < 6; q++) {
          const int pa = PA[q], pb = PB[q];
          accR[ti][tj] = mfma_bf16(Ar[ti][pa], Br[tj][pb], accR[ti][tj]);
          accR[ti][tj] = mfma_bf16(An[ti][pa], Bi[tj][pb], accR[ti][tj]);
          accI[ti][tj] = mfma_bf16(Ar[ti][pa], Bi[tj][pb], accI[ti][tj]);
          accI[ti][tj] = mfma_bf16(Ai[ti][pa], Br[tj][pb], accI[ti][tj]);
        }
  }
}

// Output coordinates of accumulator entry e (0..3) of tile (ti, tj) for this lane.
__device__ __forceinline__ void cmma_coord(int wave, int lane, int ti, int tj, int e, int &row,
                                           int &col) {
  row = (wave >> 1) * 32 + ti * 16 + 4 * (lane >> 4) + e;
  col = (wave & 1) * 32 + tj * 16 + (lane & 15);
}

}  // namespace tn
