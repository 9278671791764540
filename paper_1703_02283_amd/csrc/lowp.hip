// Low-precision storage and products: the approximate-storage regime of
// Sections III-B and IV (intermediates stored with few mantissa bits, products
// accumulated wide) mapped onto the gfx950 matrix cores.
//
//  * quantize_t: rounds a float64 matrix to bf16, fp16 or fp8 e4m3 (round to
//    nearest, ties to even, from the float64 value directly) after scaling each
//    128 x 128 tile by a power of two that puts its largest magnitude in
//    [2^top, 2^(top+1)) (none for bf16, whose range is float32's). The codes are
//    written transposed and zero padded to a multiple of 128, which is the
//    k-contiguous layout the matrix-core operands want: lane l of a 16x16x32
//    MFMA supplies 8 consecutive k of one row.
//  * gemm_lp: D = L^T R from two such operands, fp32 accumulation on
//    v_mfma_f32_16x16x32_{bf16,f16} or v_mfma_f32_16x16x32_fp8_fp8, with the
//    per-tile scales applied once per 128-wide k block, then the float64
//    epilogue shared with the FP64 kernel.
#include <cstdint>

#include "kernels_common.h"
#include "lowp.h"

namespace ipr {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));

constexpr int TILE = 128;
constexpr int NT = 256;

struct Fmt {
  int t;        // significand bits including the implicit one
  int emin;     // exponent of the smallest normal
  double vmax;  // largest finite
  int top;      // tile scaling target exponent (-1000: unscaled)
};

__host__ __device__ inline Fmt fmt_of(int dtype) {
  switch (dtype) {
    case LP_BF16: return {8, -126, 3.3895313892515355e38, -1000};
    case LP_FP16: return {11, -14, 65504.0, 14};
    default: return {4, -6, 448.0, 7};
  }
}

// Round x (already scaled) to the format, returned as an exactly representable double.
__device__ inline double round_fmt(double x, const Fmt& f) {
  if (x == 0.0) return 0.0;
  const double a = fabs(x);
  int e = ilogb(a);
  if (e < f.emin) e = f.emin;
  const double ulp = ldexp(1.0, e - (f.t - 1));
  double y = rint(a / ulp) * ulp;
  if (y > f.vmax) y = f.vmax;
  return copysign(y, x);
}

__device__ inline uint16_t bits_bf16(double y) {
  return (uint16_t)(__float_as_uint((float)y) >> 16);  // exact: y has <= 8 significant bits
}
__device__ inline uint16_t bits_fp16(double y) {
  _Float16 h = (_Float16)(float)y;                     // exact
  return *reinterpret_cast<uint16_t*>(&h);
}
__device__ inline uint8_t bits_e4m3(double y) {
  uint8_t s = y < 0 ? 0x80 : 0;
  const double a = fabs(y);
  if (a == 0.0) return s;
  const int e = ilogb(a);
  if (e < -6) return s | (uint8_t)(int)(a * 512.0);            // subnormal: a / 2^-9
  const int m = (int)(a * ldexp(1.0, 3 - e)) - 8;             // 3 fraction bits
  return s | (uint8_t)(((e + 7) << 3) | m);
}

// One workgroup per 128 x 128 input tile (tr, tc): exponent from the tile's
// largest magnitude, then codes of X^T into Q (ldq = padded order).
template <typename T>
__global__ __launch_bounds__(NT) void quantize_t_kernel(const double* __restrict__ X, int n,
                                                         int ldq, int ntp, int dtype,
                                                         T* __restrict__ Q,
                                                         int* __restrict__ E) {
  __shared__ double red[NT];
  __shared__ int sh_e;
  const int tr = blockIdx.y, tc = blockIdx.x;
  const int r0 = tr * TILE, c0 = tc * TILE;
  const Fmt f = fmt_of(dtype);
  // tile amax (row-major reads, coalesced)
  double m = 0.0;
  for (int t = threadIdx.x; t < TILE * TILE; t += NT) {
    const int r = r0 + t / TILE, c = c0 + t % TILE;
    if (r < n && c < n) m = fmax(m, fabs(X[(size_t)r * n + c]));
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    int e = 0;
    if (f.top > -1000 && red[0] > 0.0) e = ilogb(red[0]) - f.top;
    sh_e = e;
    E[tc * ntp + tr] = e;   // transposed tile index, like the codes
  }
  __syncthreads();
  const double scale = ldexp(1.0, -sh_e);
  // transposed write: output row c (input column), 128 consecutive r.
  // thread t handles output row c0 + t/2, r in [r0 + 64 (t%2), +64)
  const int c = c0 + (threadIdx.x >> 1);
  const int rb = r0 + 64 * (threadIdx.x & 1);
  T* qrow = Q + (size_t)c * ldq;
  for (int rr = 0; rr < 64; ++rr) {
    const int r = rb + rr;
    double v = (r < n && c < n) ? X[(size_t)r * n + c] * scale : 0.0;
    const double y = round_fmt(v, f);
    T code;
    if constexpr (sizeof(T) == 2)
      code = dtype == LP_BF16 ? bits_bf16(y) : bits_fp16(y);
    else
      code = bits_e4m3(y);
    qrow[r] = code;
  }
}

// D = L^T R from k-contiguous codes Lt (row i), Rt (row j), order np (multiple of 128).
// ESZ = bytes per code. 4 waves (2 x 2) x 64 x 64 per wave.
constexpr int ROWB = 128;        // bytes of k per LDS row and stage
constexpr int PITCH = ROWB + 16; // LDS row pitch in bytes

template <int ESZ, int DT>
__global__ __launch_bounds__(NT, 2) void gemm_lp_kernel(const uint8_t* __restrict__ Lt,
                                                        const uint8_t* __restrict__ Rt,
                                                        const int* __restrict__ EL,
                                                        const int* __restrict__ ER, int n,
                                                        int np, Grid gr, int tri, Epilogue e) {
  __shared__ __attribute__((aligned(16))) uint8_t As[2][TILE * PITCH];
  __shared__ __attribute__((aligned(16))) uint8_t Bs[2][TILE * PITCH];
  __shared__ double red[NT / 64];
  constexpr int BKE = ROWB / ESZ;             // k elements per stage
  constexpr int KSTEPS = BKE / 32;            // MFMA k steps (32 each) per stage
  constexpr int STAGES_PER_SCALE = TILE / BKE;
  constexpr bool SCALED = DT != LP_BF16;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int lw = logical_wg();
  int bi, bj;
  if (!tile_of(lw, gr, tri, &bi, &bj)) {
    if (e.partial && tid == 0) e.partial[lw] = 0.0;
    return;
  }
  const int i0 = bi * TILE, j0 = bj * TILE;
  const int wm0 = (wave >> 1) * 64, wn0 = (wave & 1) * 64;
  const int ntp = np / TILE;

  v4f acc[4][4], blk[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      acc[a][b] = (v4f){0.f, 0.f, 0.f, 0.f};
      blk[a][b] = (v4f){0.f, 0.f, 0.f, 0.f};
    }

  // loader: 128 rows x 128 bytes per operand = 1024 chunks of 16 B; thread t
  // moves rows (t / 8) + 32 q, bytes 16 (t % 8).
  const int lrow = tid >> 3, lcb = (tid & 7) * 16;
  uint4 ga[4], gb[4];
  auto gload = [&](int kb) {  // kb = first k byte
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = lrow + 32 * q;
      ga[q] = *reinterpret_cast<const uint4*>(Lt + (size_t)(i0 + r) * np * ESZ + kb + lcb);
      gb[q] = *reinterpret_cast<const uint4*>(Rt + (size_t)(j0 + r) * np * ESZ + kb + lcb);
    }
  };
  auto lstore = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = lrow + 32 * q;
      *reinterpret_cast<uint4*>(&As[buf][r * PITCH + lcb]) = ga[q];
      *reinterpret_cast<uint4*>(&Bs[buf][r * PITCH + lcb]) = gb[q];
    }
  };

  const int nstage = np * ESZ / ROWB;
  gload(0);
  lstore(0);
  __syncthreads();
  const int fr = lane >> 4, fc = lane & 15;
  for (int st = 0; st < nstage; ++st) {
    const int buf = st & 1;
    if (st + 1 < nstage) gload((st + 1) * ROWB);
#pragma unroll
    for (int ks = 0; ks < KSTEPS; ++ks) {
      const int kbyte = (ks * 32 + fr * 8) * ESZ;
      if constexpr (ESZ == 2) {
        v8bf abf[4], bbf[4];
        v8h ah[4], bh[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          uint4 v = *reinterpret_cast<const uint4*>(&As[buf][(wm0 + a * 16 + fc) * PITCH + kbyte]);
          if constexpr (DT == LP_BF16) abf[a] = __builtin_bit_cast(v8bf, v);
          else ah[a] = __builtin_bit_cast(v8h, v);
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          uint4 v = *reinterpret_cast<const uint4*>(&Bs[buf][(wn0 + b * 16 + fc) * PITCH + kbyte]);
          if constexpr (DT == LP_BF16) bbf[b] = __builtin_bit_cast(v8bf, v);
          else bh[b] = __builtin_bit_cast(v8h, v);
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            if constexpr (DT == LP_BF16)
              blk[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(abf[a], bbf[b], blk[a][b], 0, 0, 0);
            else
              blk[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[a], bh[b], blk[a][b], 0, 0, 0);
          }
      } else {
        long a8[4], b8[4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
          a8[a] = *reinterpret_cast<const long*>(&As[buf][(wm0 + a * 16 + fc) * PITCH + kbyte]);
#pragma unroll
        for (int b = 0; b < 4; ++b)
          b8[b] = *reinterpret_cast<const long*>(&Bs[buf][(wn0 + b * 16 + fc) * PITCH + kbyte]);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b)
            blk[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(a8[a], b8[b], blk[a][b], 0, 0, 0);
      }
    }
    if constexpr (SCALED) {
      if ((st + 1) % STAGES_PER_SCALE == 0) {
        const int kt = st / STAGES_PER_SCALE;
        const float sc = ldexpf(1.0f, EL[bi * ntp + kt] + ER[bj * ntp + kt]);
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            acc[a][b] += sc * blk[a][b];
            blk[a][b] = (v4f){0.f, 0.f, 0.f, 0.f};
          }
      }
    }
    if (st + 1 < nstage) lstore(buf ^ 1);
    __syncthreads();
  }
  // f32 16x16 output layout: row 4 (lane / 16) + r, column lane % 16
  double psum = 0.0;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float v = SCALED ? acc[a][b][r] : blk[a][b][r];
        epilogue_element(e, n, tri, i0 + wm0 + a * 16 + 4 * fr + r, j0 + wn0 + b * 16 + fc,
                         (double)v, psum);
      }
  if (e.partial) store_partial(e.partial, lw, psum, red);
}

}  // namespace

int lp_padded(int n) { return (n + TILE - 1) / TILE * TILE; }
int lp_esize(int dtype) { return dtype == LP_FP8 ? 1 : 2; }
size_t lp_bytes(int n, int dtype) {
  const size_t np = lp_padded(n);
  return np * np * lp_esize(dtype);
}
size_t lp_exp_count(int n) {
  const size_t t = lp_padded(n) / TILE;
  return t * t;
}
int lp_partial_slots(int n, int tri) { return make_grid(n, tri, TILE).nwg; }

hipError_t quantize_t(const double* X, int n, int dtype, void* Q, int* E, hipStream_t stream) {
  const int np = lp_padded(n), ntp = np / TILE;
  dim3 grid(ntp, ntp);
  if (lp_esize(dtype) == 2)
    hipLaunchKernelGGL(quantize_t_kernel<uint16_t>, grid, dim3(NT), 0, stream, X, n, np, ntp,
                       dtype, (uint16_t*)Q, E);
  else
    hipLaunchKernelGGL(quantize_t_kernel<uint8_t>, grid, dim3(NT), 0, stream, X, n, np, ntp,
                       dtype, (uint8_t*)Q, E);
  return hipGetLastError();
}

hipError_t gemm_lp(const void* Lq, const int* EL, const void* Rq, const int* ER, int n,
                   int dtype, int tri, const Epilogue& e, hipStream_t stream) {
  if (!Lq || !Rq || !EL || !ER) return hipErrorInvalidValue;
  const int np = lp_padded(n);
  // tiles beyond n are empty: grid over the unpadded order
  Grid gr = make_grid(n, tri, TILE);
  const uint8_t* L = (const uint8_t*)Lq;
  const uint8_t* R = (const uint8_t*)Rq;
  switch (dtype) {
    case LP_BF16:
      hipLaunchKernelGGL((gemm_lp_kernel<2, LP_BF16>), dim3(gr.nwg), dim3(NT), 0, stream, L, R,
                         EL, ER, n, np, gr, tri, e);
      break;
    case LP_FP16:
      hipLaunchKernelGGL((gemm_lp_kernel<2, LP_FP16>), dim3(gr.nwg), dim3(NT), 0, stream, L, R,
                         EL, ER, n, np, gr, tri, e);
      break;
    default:
      hipLaunchKernelGGL((gemm_lp_kernel<1, LP_FP8>), dim3(gr.nwg), dim3(NT), 0, stream, L, R,
                         EL, ER, n, np, gr, tri, e);
  }
  return hipGetLastError();
}

}  // namespace ipr
