// Low-precision storage and products: the approximate-storage regime of
// Sections III-B and IV (intermediates stored with few mantissa bits, products
// accumulated wide) mapped onto the gfx950 matrix cores.
//
//  * quantize_t: rounds a float64 matrix to bf16, fp16 or fp8 e4m3 (round to
//    nearest, ties to even, from the float64 value directly) after scaling each
//    128 x 128 tile by a power of two that puts its largest magnitude in
//    [2^top, 2^(top+1)) (none for bf16, whose range is float32's). The codes are
//    written transposed and zero padded to a multiple of 256, which is the
//    k-contiguous layout the matrix-core operands want (a lane supplies 8 or 32
//    consecutive k of one row).
//  * gemm_lp: D = L^T R from two such operands on the matrix cores with fp32
//    accumulation, then the float64 epilogue shared with the FP64 kernel
//    (details at the kernel).
//  * slices_split / gemm_slices: FP64-accurate products from int8 digit
//    slices (error-free splitting), the same kernel with int8 operands and
//    exact int32 accumulation, one launch per level of digit pairs (details
//    above colmax_kernel).
#include <algorithm>
#include <cstdint>

#include "kernels_common.h"
#include "lowp.h"

namespace ipr {
namespace {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

constexpr int TILE = 128;
constexpr int kZeroTile = -(1 << 20);   // exponent of an all-zero tile
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

constexpr int BT = 256;                 // output tile edge
constexpr int KB = 64;                  // bytes of k per row and stage
constexpr int NSTG = 4;                 // LDS ring depth
constexpr int STG_BYTES = BT * KB;      // one operand, one stage

// Physical chunk of logical 16-byte chunk `chunk` in LDS row `row`. Any 8
// consecutive rows read at one logical chunk cover a 128-byte period, and
// any 16 a 256-byte period, without two lanes on one bank.
__device__ __forceinline__ int swz(int row, int chunk) {
  return chunk ^ ((row >> 1) & 3) ^ (((row >> 3) & 1) * 3);
}

// Byte offset of the 16-byte piece of row i that starts at byte kb of the
// row, in the blocked layout of the codes: for each 256-row block and each
// 64-byte stage of k, the 256 x 64 bytes the product kernel moves into LDS
// for that stage are stored contiguously and in LDS order (rows of 4 chunks,
// swizzled), so a wave's load is one contiguous kilobyte.
__host__ __device__ inline size_t lp_block_offset(int i, int kb, int nst) {
  const int r = i % BT, c = (kb % KB) / 16;
  return ((size_t)(i / BT) * nst + kb / KB) * (size_t)(BT * KB) + (size_t)r * KB + 16 * swz(r, c);
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
  __shared__ __attribute__((aligned(16))) T cT[TILE][TILE + 2];   // codes, transposed
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
    // an all-zero tile gets kZeroTile, which the product kernel skips
    int e = kZeroTile;
    if (red[0] > 0.0) e = f.top > -1000 ? ilogb(red[0]) - f.top : 0;
    sh_e = e == kZeroTile ? 0 : e;
    E[tc * ntp + tr] = e;   // transposed tile index, like the codes
  }
  __syncthreads();
  const double scale = ldexp(1.0, -sh_e);
  // codes in input order (coalesced reads of X; the tile is L2-resident from
  // the pass above) into LDS, transposed: cT[c][r]
  for (int t = threadIdx.x; t < TILE * TILE; t += NT) {
    const int rl = t / TILE, cl = t % TILE;
    const int r = r0 + rl, c = c0 + cl;
    const double v = (r < n && c < n) ? X[(size_t)r * n + c] * scale : 0.0;
    const double y = round_fmt(v, f);
    T code;
    if constexpr (sizeof(T) == 2)
      code = dtype == LP_BF16 ? bits_bf16(y) : bits_fp16(y);
    else
      code = bits_e4m3(y);
    cT[cl][rl] = code;
  }
  __syncthreads();
  // rows of Q (= columns of X) in 16-byte pieces: consecutive threads write
  // consecutive pieces of a row
  constexpr int PER = 16 / sizeof(T);          // codes per piece
  constexpr int PIECES = TILE / PER;           // pieces per row
  for (int t = threadIdx.x; t < TILE * PIECES; t += NT) {
    const int cl = t / PIECES, pc = t % PIECES;
    const T* src = &cT[cl][pc * PER];
    uint32_t wd[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      if constexpr (sizeof(T) == 2)
        wd[k] = (uint32_t)src[2 * k] | ((uint32_t)src[2 * k + 1] << 16);
      else
        wd[k] = (uint32_t)src[4 * k] | ((uint32_t)src[4 * k + 1] << 8) |
                ((uint32_t)src[4 * k + 2] << 16) | ((uint32_t)src[4 * k + 3] << 24);
    }
    const int nst = ldq * (int)sizeof(T) / KB;
    *reinterpret_cast<uint4*>(reinterpret_cast<uint8_t*>(Q) +
                              lp_block_offset(c0 + cl, (r0 + pc * PER) * (int)sizeof(T), nst)) =
        make_uint4(wd[0], wd[1], wd[2], wd[3]);
  }
}

// One launch of the int8-slice product covers one chunk of the pairs (t, u)
// of one level g = t + u (see gemm_slices): digit slices t of L^T and u of
// R^T, concatenated along k, accumulate exactly in int32.
struct SliceArgs {
  int npairs;               // pairs in this chunk
  unsigned long long tpk;   // slice index of L^T for pair q in bits 4q .. 4q + 3
  unsigned long long upk;   // same for R^T
  size_t slice_bytes;       // bytes of one digit matrix
  double* P;                // exact partial sum of a level split into chunks
  double* S;                // running float64 sum of the finished levels
  int first_chunk, last_chunk, first_level, final_level;
  int shift;                // beta g
};

constexpr int kNonFinite = 0x7fffffff;  // row exponent of a row holding Inf or NaN

// Element (i, j) of a chunk's int32 result iv, with the values already read
// from P (pv: the level's exact partial sum) and S (sv: the running sum):
// exact level sum, then the scaled level added to the running sum (smallest
// level first); the last level goes through the product epilogue.
__device__ __forceinline__ void slice_element(const SliceArgs& sa, const int* EL, const int* ER,
                                              const Epilogue& e, int n, int tri, int i, int j,
                                              int iv, double pv, double sv, double& psum) {
  if (i >= n || j >= n) return;
  const size_t ij = (size_t)i * n + j;
  double v = (double)iv;
  if (!sa.first_chunk) v += pv;   // integers below 2^53: exact
  if (!sa.last_chunk) {
    sa.P[ij] = v;
    return;
  }
  const int ei = EL[i], ej = ER[j];
  double term = (ei == kNonFinite || ej == kNonFinite) ? __builtin_nan("")
                                                       : ldexp(v, ei + ej - sa.shift);
  if (!sa.first_level) term = sv + term;
  if (!sa.final_level) {
    sa.S[ij] = term;
    return;
  }
  epilogue_element<false>(e, n, tri, i, j, term, psum);
}

// D = L^T R from k-contiguous codes Lt (row i), Rt (row j), order np (a
// multiple of 256), on 256 x 256 output tiles.
//
// * 4 waves (2 x 2), each a 128 x 128 sub-tile = 4 x 4 blocks of 32 x 32
//   (v_mfma_f32_32x32x16_{bf16,f16}: lane l supplies row l % 32, k 8 (l / 32)
//   .. + 7; v_mfma_scale_f32_32x32x64_f8f6f4 for fp8: k 32 (l / 32) .. + 31).
//   A wave's 128 rows and columns are one 128 x 128 exponent tile each.
// * k is staged 64 bytes per row at a time through a ring of NSTG LDS buffers
//   filled by direct global -> LDS loads (16 bytes per lane, the lane's data
//   lands at base + 16 lane), NSTG - 1 stages ahead of the matrix cores. In
//   LDS a row is 4 chunks of 16 bytes, chunk c of row r stored at c ^ ((r / 2)
//   & 3): the fragment reads of 8 consecutive rows then hit distinct banks.
// * Per-tile exponents: fp8 passes them to the matrix core as block scales
//   (E8M0 127 + e, exact). fp16 keeps the accumulator in units of 2^Sref,
//   Sref = max over k-tiles of eL + eR for the wave's exponent tiles, and
//   multiplies the A fragments of k-tile t by 2^(eL + eR - Sref) <= 1 (exact
//   unless it underflows fp16, i.e. below 2^-24 of the largest k-tile's scale).
//   bf16 is unscaled.
typedef float v16f __attribute__((ext_vector_type(16)));
typedef int v8i __attribute__((ext_vector_type(8)));
typedef __attribute__((address_space(3))) void lds_void;

template <int V>
struct Ic {
  static constexpr int value = V;
};

// A compiler-only fence: keeps LDS reads and writes on their side of a
// barrier without the hardware wait that __syncthreads adds for every
// outstanding load (the ring's loads of later stages must stay in flight).
__device__ __forceinline__ void wg_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

template <int ESZ, int DT>
__global__ __launch_bounds__(NT, 1) void gemm_lp_kernel(const uint8_t* __restrict__ Lt,
                                                        const uint8_t* __restrict__ Rt,
                                                        const int* __restrict__ EL,
                                                        const int* __restrict__ ER, int n,
                                                        int np, Grid gr, int tri, Epilogue e,
                                                        SliceArgs sa) {
  // one array per ring slot: distinct objects let the compiler see that the
  // loads in flight into other slots do not alias the slot being read
  __shared__ __attribute__((aligned(16))) uint8_t A0[STG_BYTES], A1[STG_BYTES], A2[STG_BYTES],
      A3[STG_BYTES];
  __shared__ __attribute__((aligned(16))) uint8_t B0[STG_BYTES], B1[STG_BYTES], B2[STG_BYTES],
      B3[STG_BYTES];
  __shared__ double red[NT / 64];
  __shared__ double post_sh[4];             // per wave: fp16 result scale 2^Sref
  constexpr int KEL = KB / ESZ;             // k elements per stage
  constexpr int ST_PER_KT = TILE / KEL;     // stages per 128-wide exponent tile
  static_assert(NSTG == 4, "four ring slots");

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  // Persistent: one workgroup per CU; the workgroups of an XCD (w % 8) walk
  // that XCD's run of logical tiles together, 32 consecutive tiles at a time,
  // so their row and column panels are read from its L2 at about the same k.
  const int per = gr.nwg >> 3;            // logical tiles per XCD
  const int nx = gridDim.x >> 3;          // workgroups per XCD
  const int xcd = blockIdx.x & 7;
  for (int t = blockIdx.x >> 3; t < per; t += nx) {
  const int lw = xcd * per + t;
  int bi, bj;
  if (!tile_of(lw, gr, tri, &bi, &bj)) {
    if (e.partial && tid == 0) e.partial[lw] = 0.0;
    continue;
  }
  wg_barrier();  // the previous tile's epilogue is done with the LDS
  const int i0 = bi * BT, j0 = bj * BT;
  const int wm = wave >> 1, wn = wave & 1;
  const int ntp = np / TILE;
  const int ib = 2 * bi + wm, jb = 2 * bj + wn;   // the wave's exponent tiles
  const size_t ldb = (size_t)np * ESZ;

  // exponent reference (fp16)
  int sref = 0;
  if constexpr (DT == LP_FP16) {
    sref = kZeroTile;   // stays so only when every product of tiles is zero
    for (int kt = 0; kt < ntp; ++kt) {
      const int el = EL[ib * ntp + kt], er = ER[jb * ntp + kt];
      if (el == kZeroTile || er == kZeroTile) continue;
      sref = el + er > sref ? el + er : sref;
    }
  }

  // loader: instruction q of wave w fills rows 64 w + 16 q .. + 15 of a stage;
  // lane l's 16 bytes land at row (l / 4), physical chunk l % 4
  // the blocked layout holds each stage's 256 x 64 bytes contiguously and in
  // LDS order: lane l of instruction q copies bytes (64 w + 16 q) 64 + 16 l
  const int nst_all = (int)(ldb / KB);
  const int nst1 = nst_all;   // stages per operand pair
  const uint8_t* gA[4];
  const uint8_t* gB[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const size_t in_block = (size_t)(64 * wave + 16 * q) * KB + 16 * lane;
    gA[q] = Lt + (size_t)bi * nst_all * (BT * KB) + in_block;
    gB[q] = Rt + (size_t)bj * nst_all * (BT * KB) + in_block;
  }
  auto issue = [&](auto S, int st) {
    constexpr int sl = decltype(S)::value;
    uint8_t* as = sl == 0 ? A0 : sl == 1 ? A1 : sl == 2 ? A2 : A3;
    uint8_t* bs = sl == 0 ? B0 : sl == 1 ? B1 : sl == 2 ? B2 : B3;
    size_t ka0, kb0;   // stage st's block of each operand
    if constexpr (DT == LP_I8) {
      const int pr = st / nst1;   // pair
      const size_t off = (size_t)(st - pr * nst1) * (BT * KB);
      ka0 = off + (size_t)((sa.tpk >> (4 * pr)) & 15) * sa.slice_bytes;
      kb0 = off + (size_t)((sa.upk >> (4 * pr)) & 15) * sa.slice_bytes;
    } else {
      ka0 = kb0 = (size_t)st * (BT * KB);
    }
    // LDS destinations as plain addresses (wave-uniform, in scalar registers)
    const uint32_t la = __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(lds_void*)as);
    const uint32_t lb = __builtin_amdgcn_readfirstlane((uint32_t)(uintptr_t)(lds_void*)bs);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint32_t off = (64 * wave + 16 * q) * KB;
      __builtin_amdgcn_global_load_lds((const void*)(gA[q] + ka0), (lds_void*)(uintptr_t)(la + off),
                                       16, 0, 0);
      __builtin_amdgcn_global_load_lds((const void*)(gB[q] + kb0), (lds_void*)(uintptr_t)(lb + off),
                                       16, 0, 0);
    }
  };

  v16f acc[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[a][b][r] = 0.f;

  const int frow = lane & 31, fhalf = lane >> 5;
  auto compute = [&](auto S, int st) {
    constexpr int sl = decltype(S)::value;
    const uint8_t* as = sl == 0 ? A0 : sl == 1 ? A1 : sl == 2 ? A2 : A3;
    const uint8_t* bs = sl == 0 ? B0 : sl == 1 ? B1 : sl == 2 ? B2 : B3;
    const int kt = st / ST_PER_KT;
    if constexpr (ESZ == 2 || DT == LP_I8) {
      _Float16 fsc = (_Float16)1.0f;
      bool scale_a = false;
      if constexpr (DT == LP_FP16) {
        const int el = EL[ib * ntp + kt], er = ER[jb * ntp + kt];
        // (a zero tile's codes are zero: any scale will do)
        const int d = (el == kZeroTile || er == kZeroTile) ? 0 : el + er - sref;
        scale_a = d != 0;
        fsc = (_Float16)ldexpf(1.0f, d < -30 ? -30 : d);
      }
      // fragments of k-step ks + 1 are read while the matrix cores work on
      // k-step ks (two MFMAs per LDS read)
      auto load = [&](int ks, uint4* av, uint4* bv) {
        const int c = 2 * ks + fhalf;
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const int row = wm * 128 + a * 32 + frow;
          av[a] = *reinterpret_cast<const uint4*>(as + row * KB + 16 * swz(row, c));
        }
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          const int row = wn * 128 + b * 32 + frow;
          bv[b] = *reinterpret_cast<const uint4*>(bs + row * KB + 16 * swz(row, c));
        }
      };
      uint4 av[2][4], bv[2][4];
      load(0, av[0], bv[0]);
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int ks = 0; ks < KB / 32; ++ks) {
        const int cur = ks & 1;
        if (ks + 1 < KB / 32) load(ks + 1, av[cur ^ 1], bv[cur ^ 1]);
        if constexpr (DT == LP_FP16) {
          if (scale_a) {
#pragma unroll
            for (int a = 0; a < 4; ++a) {
              v8h h = __builtin_bit_cast(v8h, av[cur][a]);
              h = h * fsc;
              av[cur][a] = __builtin_bit_cast(uint4, h);
            }
          }
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
          for (int b = 0; b < 4; ++b) {
            if constexpr (DT == LP_BF16)
              acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                  __builtin_bit_cast(v8bf, av[cur][a]), __builtin_bit_cast(v8bf, bv[cur][b]),
                  acc[a][b], 0, 0, 0);
            else if constexpr (DT == LP_I8)
              // int32 results kept in the float accumulators' registers as bits
              acc[a][b] = __builtin_bit_cast(
                  v16f, __builtin_amdgcn_mfma_i32_32x32x32_i8(
                            __builtin_bit_cast(v4i, av[cur][a]), __builtin_bit_cast(v4i, bv[cur][b]),
                            __builtin_bit_cast(v16i, acc[a][b]), 0, 0, 0));
            else
              acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                  __builtin_bit_cast(v8h, av[cur][a]), __builtin_bit_cast(v8h, bv[cur][b]),
                  acc[a][b], 0, 0, 0);
          }
        if constexpr (DT == LP_BF16 || DT == LP_I8) {
          if (ks + 1 < KB / 32) {
#pragma unroll
            for (int g = 0; g < 8; ++g) {
              __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);  // 2 MFMA
              __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // 1 DS read
            }
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    } else {
      // fp8: one 64-k step per stage, 32 bytes (two chunks) per lane
      // E8M0 block scales; tiles beyond float32's range clamp (they cannot
      // be accumulated in float32 anyway)
      const int sa = min(254, max(1, 127 + EL[ib * ntp + kt]));
      const int sb = min(254, max(1, 127 + ER[jb * ntp + kt]));
      v8i av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int row = wm * 128 + a * 32 + frow;
        const uint4 lo = *reinterpret_cast<const uint4*>(as + row * KB + 16 * swz(row, 2 * fhalf));
        const uint4 hi =
            *reinterpret_cast<const uint4*>(as + row * KB + 16 * swz(row, 2 * fhalf + 1));
        av[a] = (v8i){(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w,
                      (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
      }
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int row = wn * 128 + b * 32 + frow;
        const uint4 lo = *reinterpret_cast<const uint4*>(bs + row * KB + 16 * swz(row, 2 * fhalf));
        const uint4 hi =
            *reinterpret_cast<const uint4*>(bs + row * KB + 16 * swz(row, 2 * fhalf + 1));
        bv[b] = (v8i){(int)lo.x, (int)lo.y, (int)lo.z, (int)lo.w,
                      (int)hi.x, (int)hi.y, (int)hi.z, (int)hi.w};
      }
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(av[a], bv[b], acc[a][b], 0,
                                                                      0, 0, sa, 0, sb);
    }
  };

  // (s_waitcnt fields: vmcnt bits 3:0 and 15:14, expcnt 6:4 = 7, lgkmcnt
  // 11:8 = 15, i.e. only the vector-memory count is waited on; a stage is 8
  // loads per lane)
  auto stage = [&](auto S, int st, int nst) {
    constexpr int sl = decltype(S)::value;
    const int after = nst - 1 - st;   // stages issued after st (at most 2)
    if (after >= 2) __builtin_amdgcn_s_waitcnt(0x4F70);       // vmcnt(16)
    else if (after == 1) __builtin_amdgcn_s_waitcnt(0x0F78);  // vmcnt(8)
    else __builtin_amdgcn_s_waitcnt(0x0F70);                  // vmcnt(0)
    wg_barrier();  // stage st is in LDS for every wave; slot (st + 3) % 4 is free
    if (st + 3 < nst) issue(Ic<(sl + 3) % 4>{}, st + 3);
    compute(S, st);
  };

  // a multiple of 4 (np is a multiple of 256)
  const int nst = (int)(ldb / KB) * (DT == LP_I8 ? sa.npairs : 1);
  auto wait_stage = [&](int st) {
    const int after = nst - 1 - st;   // stages issued after st (at most 2)
    if (after >= 2) __builtin_amdgcn_s_waitcnt(0x4F70);       // vmcnt(16)
    else if (after == 1) __builtin_amdgcn_s_waitcnt(0x0F78);  // vmcnt(8)
    else __builtin_amdgcn_s_waitcnt(0x0F70);                  // vmcnt(0)
  };
  issue(Ic<0>{}, 0);
  issue(Ic<1>{}, 1);
  issue(Ic<2>{}, 2);
  if constexpr (ESZ == 2 || DT == LP_I8) {
    // Two k-steps per stage. The barrier of stage st + 1 sits before the
    // last k-step of stage st: by then each wave holds that step's
    // fragments (it waits for its LDS reads first), so the slot can be
    // refilled right after the barrier, and the first fragments of stage
    // st + 1 are read from LDS between the last step's MFMAs (no LDS latency
    // exposed at the stage boundary).
    static_assert(KB / 32 == 2, "two k-steps per stage");
    auto frag = [&](auto S, int ks, uint4* av, uint4* bv) {
      constexpr int sl = decltype(S)::value;
      const uint8_t* as = sl == 0 ? A0 : sl == 1 ? A1 : sl == 2 ? A2 : A3;
      const uint8_t* bs = sl == 0 ? B0 : sl == 1 ? B1 : sl == 2 ? B2 : B3;
      const int c = 2 * ks + fhalf;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const int row = wm * 128 + a * 32 + frow;
        av[a] = *reinterpret_cast<const uint4*>(as + row * KB + 16 * swz(row, c));
      }
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int row = wn * 128 + b * 32 + frow;
        bv[b] = *reinterpret_cast<const uint4*>(bs + row * KB + 16 * swz(row, c));
      }
    };
    auto mfmas = [&](const uint4* av, const uint4* bv) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          if constexpr (DT == LP_BF16)
            acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                __builtin_bit_cast(v8bf, av[a]), __builtin_bit_cast(v8bf, bv[b]), acc[a][b], 0, 0,
                0);
          else if constexpr (DT == LP_I8)
            // int32 results kept in the float accumulators' registers as bits
            acc[a][b] = __builtin_bit_cast(
                v16f, __builtin_amdgcn_mfma_i32_32x32x32_i8(
                          __builtin_bit_cast(v4i, av[a]), __builtin_bit_cast(v4i, bv[b]),
                          __builtin_bit_cast(v16i, acc[a][b]), 0, 0, 0));
          else
            acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_f16(
                __builtin_bit_cast(v8h, av[a]), __builtin_bit_cast(v8h, bv[b]), acc[a][b], 0, 0,
                0);
        }
#pragma unroll
      for (int g = 0; g < 8; ++g) {
        __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);  // 2 MFMA
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // 1 DS read
      }
    };
    // fp16: stage st's fragments of A rescaled to the accumulator's units
    auto rescale = [&](int st, uint4* av) {
      if constexpr (DT == LP_FP16) {
        const int kt = st / ST_PER_KT;
        const int el = EL[ib * ntp + kt], er = ER[jb * ntp + kt];
        // (a zero tile's codes are zero: any scale will do)
        const int d = (el == kZeroTile || er == kZeroTile) ? 0 : el + er - sref;
        if (d != 0) {
          const _Float16 fsc = (_Float16)ldexpf(1.0f, d < -30 ? -30 : d);
#pragma unroll
          for (int a = 0; a < 4; ++a) {
            v8h h = __builtin_bit_cast(v8h, av[a]);
            h = h * fsc;
            av[a] = __builtin_bit_cast(uint4, h);
          }
        }
      }
    };
    uint4 av[2][4], bv[2][4];
    auto step = [&](auto S, int st) {
      constexpr int sl = decltype(S)::value;
      // k-step 0 of stage st (fragments in av[0]); k-step 1's are read meanwhile
      frag(S, 1, av[1], bv[1]);
      rescale(st, av[0]);
      mfmas(av[0], bv[0]);
      __builtin_amdgcn_sched_barrier(0);
      // k-step 1; the barrier of stage st + 1 first (after the last stage the
      // same steps run on no data: the wait is for every load, and the
      // fragments read are not used)
      __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): k-step 1's fragments are in
      wait_stage(st + 1);
      wg_barrier();  // stage st + 1 is in LDS for every wave; this slot is free
      if (st + 4 < nst) issue(S, st + 4);
      __builtin_amdgcn_sched_barrier(0);
      frag(Ic<(sl + 1) % 4>{}, 0, av[0], bv[0]);
      rescale(st, av[1]);
      mfmas(av[1], bv[1]);
      __builtin_amdgcn_sched_barrier(0);
    };
    wait_stage(0);
    wg_barrier();
    issue(Ic<3>{}, 3);
    frag(Ic<0>{}, 0, av[0], bv[0]);
    for (int st = 0; st < nst; st += 4) {
      step(Ic<0>{}, st);
      step(Ic<1>{}, st + 1);
      step(Ic<2>{}, st + 2);
      step(Ic<3>{}, st + 3);
    }
  } else {
    for (int st = 0; st < nst; st += 4) {
      stage(Ic<0>{}, st, nst);
      stage(Ic<1>{}, st + 1, nst);
      stage(Ic<2>{}, st + 2, nst);
      stage(Ic<3>{}, st + 3, nst);
    }
  }

  // Epilogue through LDS, one 32-row block of each wave at a time: the waves
  // write their fp32 results row-major into a 64 x 256 staging area (the ring
  // slots), then thread t takes column t of the 64 rows.
  // 32 x 32 f32 output layout: register r of lane l is row (r % 4) + 8 (r / 4)
  // + 4 (l / 32), column l % 32.
  // the staging area holds each wave's results in its own units (fp16: 2^Sref)
  if (lane == 0)
    post_sh[wave] = DT != LP_FP16 ? 1.0 : sref == kZeroTile ? 0.0 : ldexp(1.0, sref);
  double psum = 0.0;
  auto stg_at = [&](int row, int col) -> float* {
    // rows 0..15 in A0, 16..31 in A1, 32..47 in A2, 48..63 in A3 (16 KB each)
    float* base = reinterpret_cast<float*>(row < 16 ? A0 : row < 32 ? A1 : row < 48 ? A2 : A3);
    return base + (row & 15) * 256 + col;
  };
#pragma unroll
  for (int h = 0; h < 4; ++h) {
    wg_barrier();  // previous users of the staging area are done
#pragma unroll
    for (int b = 0; b < 4; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = wm * 32 + (r & 3) + 8 * (r >> 2) + 4 * fhalf;
        const int col = wn * 128 + b * 32 + frow;
        // (int8 products: the int32 bits travel as a float, moved, never computed on)
        *stg_at(row, col) = acc[h][b][r];
      }
    wg_barrier();
    if constexpr (DT == LP_I8) {
      // the partial and running sums of 16 rows are read before any is
      // written: the stores may alias the loads as far as the compiler
      // knows, and one round trip to memory per element would serialise
      const bool need_p = !sa.first_chunk, need_s = sa.last_chunk && !sa.first_level;
      const int j = j0 + tid;
      for (int q0 = 0; q0 < 64; q0 += 16) {
        double pv[16], sv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int q = q0 + u;
          const int i = i0 + (q >> 5) * 128 + h * 32 + (q & 31);
          const bool in = i < n && j < n;
          const size_t ij = (size_t)i * n + j;
          pv[u] = in && need_p ? sa.P[ij] : 0.0;
          sv[u] = in && need_s ? sa.S[ij] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) {
          const int q = q0 + u;
          const int i = i0 + (q >> 5) * 128 + h * 32 + (q & 31);
          slice_element(sa, EL, ER, e, n, tri, i, j, __float_as_int(*stg_at(q, tid)), pv[u],
                        sv[u], psum);
        }
      }
    } else {
      for (int q = 0; q < 64; ++q) {
        const int i = i0 + (q >> 5) * 128 + h * 32 + (q & 31);
        const int j = j0 + tid;
        const double post = post_sh[(q >> 5) * 2 + (tid >> 7)];  // the owning wave's
        epilogue_element<false>(e, n, tri, i, j, (double)*stg_at(q, tid) * post, psum);
      }
    }
  }
  if (e.partial) store_partial(e.partial, lw, psum, red);
  }
}

// ---- FP64-accurate products from int8 digit slices ----------------------
//
// Error-free splitting (Ozaki, Ogita, Oishi and Rump, Numer. Algorithms 59,
// 2012) with beta = 7-bit digits: row i of an operand is scaled by 2^-e_i,
// e_i the smallest integer above its largest magnitude's exponent, and cut
// into s digits d_t = round(2^7 r) (nearest, ties to even, clamped to
// [-127, 127]), r the remainder of the previous digit. The digit matrices
// multiply exactly on the int8 matrix cores; level g = t + u sums the pairs
// of slices (t, u), g <= s + 1, exactly in int32; the levels are scaled and
// added in float64 from the smallest to the largest.

// Largest magnitude of each column of X as the bit pattern of a double
// (non-negative doubles order like their bits); Inf and NaN count as Inf.
__global__ __launch_bounds__(NT) void colmax_kernel(const double* __restrict__ X, int n,
                                                    int rows, unsigned long long* __restrict__ cm) {
  const int c = blockIdx.x * NT + threadIdx.x;
  if (c >= n) return;
  const int r0 = blockIdx.y * rows, r1 = min(n, r0 + rows);
  double m = 0.0;
  for (int r = r0; r < r1; ++r) {
    const double a = fabs(X[(size_t)r * n + c]);
    m = a <= 1.79769313486231570815e308 ? fmax(m, a) : __builtin_inf();
  }
  atomicMax(&cm[c], (unsigned long long)__double_as_longlong(m));
}

__global__ __launch_bounds__(NT) void zero_u64_kernel(unsigned long long* __restrict__ v, int n) {
  const int i = blockIdx.x * NT + threadIdx.x;
  if (i < n) v[i] = 0ull;
}

// One workgroup per 64 x 64 tile (k rows, i columns) of X: digits of column
// i of X (= row i of the transposed operand), 16 consecutive k per thread,
// written as one 16-byte piece per slice in the blocked code layout. Covers
// the padded order np (zeros beyond n). Blocks of the first k tile also
// write the row exponents.
constexpr int SB = 64;
__global__ __launch_bounds__(NT) void split_kernel(const double* __restrict__ X, int n, int np,
                                                   int s, const unsigned long long* __restrict__ cm,
                                                   uint8_t* __restrict__ Q, size_t slice_bytes,
                                                   int* __restrict__ E) {
  __shared__ double xs[SB][SB + 1];
  const int k0 = blockIdx.y * SB, i0 = blockIdx.x * SB;
  for (int t = threadIdx.x; t < SB * SB; t += NT) {
    const int r = t / SB, c = t % SB;
    const int k = k0 + r, i = i0 + c;
    xs[r][c] = (k < n && i < n) ? X[(size_t)k * n + i] : 0.0;
  }
  __syncthreads();
  const int il = threadIdx.x >> 2, piece = threadIdx.x & 3;
  const int i = i0 + il;
  int e = 0;
  bool bad = false;
  if (i < n) {
    const double m = __longlong_as_double((long long)cm[i]);
    if (!(m <= 1.79769313486231570815e308))
      bad = true;
    else if (m > 0.0)
      e = ilogb(m) + 1;   // smallest e with m < 2^e
  }
  if (blockIdx.y == 0 && piece == 0) E[i] = bad ? kNonFinite : e;
  double r[16];
#pragma unroll
  for (int kk = 0; kk < 16; ++kk) r[kk] = bad ? 0.0 : ldexp(xs[piece * 16 + kk][il], -e);
  const size_t at = lp_block_offset(i, k0 + piece * 16, np / KB);
  for (int t = 0; t < s; ++t) {
    uint32_t w[4] = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      const double v = r[kk] * 128.0;   // exact
      const double d = fmin(127.0, fmax(-127.0, rint(v)));
      r[kk] = v - d;                    // exact
      w[kk >> 2] |= ((uint32_t)(int)d & 0xffu) << (8 * (kk & 3));
    }
    *reinterpret_cast<uint4*>(Q + (size_t)t * slice_bytes + at) = make_uint4(w[0], w[1], w[2], w[3]);
  }
}

}  // namespace

int lp_padded(int n) { return (n + BT - 1) / BT * BT; }
int lp_esize(int dtype) { return dtype == LP_FP8 ? 1 : 2; }
size_t lp_bytes(int n, int dtype) {
  const size_t np = lp_padded(n);
  return np * np * lp_esize(dtype);
}
size_t lp_exp_count(int n) {
  const size_t t = lp_padded(n) / TILE;
  return t * t;
}
int lp_partial_slots(int n, int tri) { return make_grid(n, tri, BT).nwg; }

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
  Grid gr = make_grid(n, tri, BT);
  const uint8_t* L = (const uint8_t*)Lq;
  const uint8_t* R = (const uint8_t*)Rq;
  static thread_local int ncu = 0;
  if (!ncu) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      ncu = 256;
  }
  const int grid = std::max(8, std::min(gr.nwg, ncu / 8 * 8));
  switch (dtype) {
    case LP_BF16:
      hipLaunchKernelGGL((gemm_lp_kernel<2, LP_BF16>), dim3(grid), dim3(NT), 0, stream, L, R,
                         EL, ER, n, np, gr, tri, e, SliceArgs{});
      break;
    case LP_FP16:
      hipLaunchKernelGGL((gemm_lp_kernel<2, LP_FP16>), dim3(grid), dim3(NT), 0, stream, L, R,
                         EL, ER, n, np, gr, tri, e, SliceArgs{});
      break;
    default:
      hipLaunchKernelGGL((gemm_lp_kernel<1, LP_FP8>), dim3(grid), dim3(NT), 0, stream, L, R,
                         EL, ER, n, np, gr, tri, e, SliceArgs{});
  }
  return hipGetLastError();
}

size_t slice_bytes(int n) {
  const size_t np = lp_padded(n);
  return np * np;
}

int slice_max_n() {
  // one pair of digit matrices must fit an int32 accumulation: np 127^2 < 2^31
  return (int)(2147483647ll / (127ll * 127ll) / BT * BT);
}

hipError_t slices_split(const double* X, int n, int s, void* Q, int* E, unsigned long long* cm,
                        hipStream_t stream) {
  if (!X || !Q || !E || !cm || s < 1 || s > kMaxSlices) return hipErrorInvalidValue;
  const int np = lp_padded(n);
  hipLaunchKernelGGL(zero_u64_kernel, dim3((n + NT - 1) / NT), dim3(NT), 0, stream, cm, n);
  const int rows = 256;
  hipLaunchKernelGGL(colmax_kernel, dim3((n + NT - 1) / NT, (n + rows - 1) / rows), dim3(NT), 0,
                     stream, X, n, rows, cm);
  hipLaunchKernelGGL(split_kernel, dim3(np / SB, np / SB), dim3(NT), 0, stream, X, n, np, s, cm,
                     (uint8_t*)Q, slice_bytes(n), E);
  return hipGetLastError();
}

hipError_t gemm_slices(const void* Lq, const int* EL, const void* Rq, const int* ER, int n, int s,
                       double* P, double* S, int tri, const Epilogue& e, hipStream_t stream) {
  if (!Lq || !Rq || !EL || !ER || !P || !S || s < 1 || s > kMaxSlices) return hipErrorInvalidValue;
  const int np = lp_padded(n);
  // pairs per int32 accumulation (cap np 127^2 < 2^31); a level with more
  // pairs is split into chunks whose sums meet exactly in P
  const long long cap = 2147483647ll / (127ll * 127ll * np);
  if (cap < 1) return hipErrorInvalidValue;
  Grid gr = make_grid(n, tri, BT);
  static thread_local int ncu = 0;
  if (!ncu) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      ncu = 256;
  }
  const int grid = std::max(8, std::min(gr.nwg, ncu / 8 * 8));
  const Epilogue none;
  for (int g = s + 1; g >= 2; --g) {
    const int t_lo = std::max(1, g - s), t_hi = std::min(s, g - 1);
    const int pairs = t_hi - t_lo + 1;
    const int per = (int)std::min<long long>(cap, 15);
    for (int c0 = 0; c0 < pairs; c0 += per) {
      SliceArgs sa{};
      sa.npairs = std::min(per, pairs - c0);
      for (int q = 0; q < sa.npairs; ++q) {
        const int t = t_lo + c0 + q, u = g - t;   // 1-based digit indices
        sa.tpk |= (unsigned long long)(t - 1) << (4 * q);
        sa.upk |= (unsigned long long)(u - 1) << (4 * q);
      }
      sa.slice_bytes = slice_bytes(n);
      sa.P = P;
      sa.S = S;
      sa.first_chunk = c0 == 0;
      sa.last_chunk = c0 + sa.npairs >= pairs;
      sa.first_level = g == s + 1;
      sa.final_level = g == 2;
      sa.shift = 7 * g;
      const bool fin = sa.final_level && sa.last_chunk;
      hipLaunchKernelGGL((gemm_lp_kernel<1, LP_I8>), dim3(grid), dim3(NT), 0, stream,
                         (const uint8_t*)Lq, (const uint8_t*)Rq, EL, ER, n, np, gr, tri,
                         fin ? e : none, sa);
      const hipError_t err = hipGetLastError();
      if (err != hipSuccess) return err;
    }
  }
  return hipSuccess;
}

}  // namespace ipr
