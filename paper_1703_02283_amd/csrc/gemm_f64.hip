// FP64 matrix-core product D = L^T R with a fused affine epilogue.
//
// Every step of the iteration of eq. (1) (Section II) is a dense n x n x n
// product followed by an elementwise update; this kernel is that step.
//
// Design for gfx950:
//  * 128 x 128 output tile per workgroup of 8 wave64s (2 x 4), each wave owning
//    64 x 32 = 4 x 2 blocks of v_mfma_f64_16x16x4f64; one workgroup per CU,
//    two waves per SIMD.
//  * Two-level accumulation: the matrix cores accumulate 64 consecutive k
//    (16 instructions per block) into a fresh slab accumulator, which is then
//    added to the tile's running sums with ordinary IEEE FP64 adds. A single
//    accumulator chained over all n of k loses accuracy with the chain length
//    (measured on gfx950: 6.6x the rms error of the two-level sum at n = 1024),
//    and in the iteration that error shows up as a residual floor several
//    times higher. In the interior loop the adds of a finished chain sit
//    between the first instructions of the next one, whose first product
//    starts from a zero accumulator.
//  * The left operand is read as L^T: for D = L^T R both operands stream rows
//    k of L and R, 128 contiguous doubles (1 KiB) per row and tile, so every
//    global load is a fully coalesced row segment and neither operand needs a
//    transpose on its way into LDS. Every left operand of the iteration is
//    symmetric, so L^T R = L R there.
//  * Interior tiles (n a multiple of 64): 16-row k slabs in a 4-slot LDS ring
//    (128 KiB, one workgroup per CU) filled by direct global-to-LDS loads
//    three slabs ahead; one barrier per slab. Edge tiles: 32-row slabs
//    staged through registers, double-buffered in the same LDS. Rows are
//    stored unpadded: each 16-lane row of an operand read is served on its
//    own, and a pitch of 144 doubles measured no faster.
//  * XCD-aware tile order: workgroup w runs on XCD w % 8, so w is remapped to
//    give each XCD a contiguous run of 8 x 8-tile super-tiles, whose 16 row and
//    column panels then stay in that XCD's L2 while its tiles are in flight.
//  * Triangle mode computes only tiles on or above the diagonal and mirrors
//    them: every product of the iteration is a polynomial in A, hence
//    symmetric, so this halves the work and keeps every iterate symmetric.
#include "kernels_common.h"

namespace ipr {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));

constexpr int BM = 128;        // tile edge (rows = cols)
constexpr int BK = 32;         // k slab per LDS stage
constexpr int WM = 64;         // wave tile rows
constexpr int WN = 32;         // wave tile columns
constexpr int FM = WM / 16;    // 16 x 16 blocks per wave, rows
constexpr int FN = WN / 16;    // 16 x 16 blocks per wave, columns
constexpr int LDP = BM;        // LDS row pitch in doubles (unpadded: see the header)
constexpr int NT = 512;        // threads per workgroup (8 waves)
constexpr int FLUSH = 2;       // slabs (2 x 32 = 64 k) per slab accumulator
constexpr int NQ = BK / 8;     // loader passes (8 rows of 128 per pass)
// interior tiles: k slabs of 16 rows in a ring of 4 LDS slots (the same LDS
// as the two 32-row buffers of the edge path), filled by direct loads
constexpr int BKD = 16;
constexpr int NSLOT = 2 * BK / BKD;        // 4
constexpr int DEPTH = NSLOT - 1;           // slabs in flight ahead of the one being read
constexpr int RPW = BKD / 8;               // k rows per wave and operand per slab
constexpr int LPS = 2 * RPW;               // direct loads per lane per slab
constexpr int FLUSHD = 64 / BKD;           // slabs per 64-k slab accumulator
static_assert(NSLOT * BKD == 2 * BK, "the two paths share the LDS buffers");
static_assert(DEPTH == 3 && FLUSHD == 4 && NSLOT == FLUSHD, "the interior loop is written for these");

// s_waitcnt with only the vector-memory count waited on: vmcnt in bits 3:0
// and 15:14, expcnt (6:4) = 7 and lgkmcnt (11:8) = 15 left open
template <int N>
__device__ __forceinline__ void wait_vm() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | 0x0F70);
}

typedef __attribute__((address_space(3))) void lds_void;

// compiler-only fence around a hardware barrier: no wait for loads in flight
__device__ __forceinline__ void wg_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// Triangle mode with a split tail: each XCD's run of q tiles is cut into
// qmain = a multiple of its CU count (whole rounds) and tailq leftover tiles,
// which would otherwise run as one round on tailq of its CUs. The leftover
// tiles are instead split along k into kparts ranges of klen, one workgroup
// each, whose raw sums go to `part`; tail_reduce_kernel adds them and applies
// the epilogue. q = 0: no split (the usual logical order).
struct TailArgs {
  int q;        // tiles per XCD run
  int qmain;    // tiles per run computed whole
  int tailq;    // tiles per run split along k
  int kparts;   // k ranges per split tile
  int klen;     // k per range (a multiple of 64)
  double* part; // 8 tailq kparts tiles of BM x BM sums
};

template <bool kSplit>
__global__ __launch_bounds__(NT, 1)
void gemm_f64_kernel(const double* __restrict__ L, const double* __restrict__ R, int n,
                     Grid gr, int tri, Epilogue e, TailArgs ta) {
  __shared__ double Ls[2][BK][LDP];
  __shared__ double Rs[2][BK][LDP];
  __shared__ double red[NT / 64];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  // Workgroup w runs on XCD w % 8; each XCD takes a contiguous run of the
  // logical order (in triangle mode of the tiles that exist, so that every
  // XCD gets the same number).
  int lw, kp = 0;
  if constexpr (kSplit) {
    const int jj = blockIdx.x >> 3;
    kp = jj / ta.tailq;
    lw = (blockIdx.x & 7) * ta.q + ta.qmain + jj % ta.tailq;
  } else {
    lw = ta.q ? (blockIdx.x & 7) * ta.q + (blockIdx.x >> 3) : logical_wg();
  }
  int bi, bj;
  const bool ok = tri ? lw < gr.nreal && tri_tile_of(lw, gr, &bi, &bj)
                      : tile_of(lw, gr, 0, &bi, &bj);
  if (!ok) {
    if (!kSplit && e.partial && tid == 0) e.partial[lw] = 0.0;
    return;
  }

  const int i0 = bi * BM, j0 = bj * BM;
  const int wm0 = (wave >> 2) * WM, wn0 = (wave & 3) * WN;

  v4d slab[FM][FN], sum[FM][FN];
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b) {
      slab[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
      sum[a][b] = slab[a][b];
    }

  const int fr = lane >> 4;   // k row of this lane's operand element
  const int fc = lane & 15;   // m (or n) index of this lane's operand element
  const bool cols_in = (i0 + BM <= n) && (j0 + BM <= n) && ((n & 1) == 0);

  if (kSplit && !(cols_in && n % 64 == 0)) return;  // (the host splits interior tiles only)
  if (cols_in && n % 64 == 0) {
    const int kbeg = kSplit ? kp * ta.klen : 0;    // first k of this workgroup's range
    // Interior tile: each wave moves RPW k rows of L and R per slab straight
    // into LDS (64 lanes x 16 bytes = one 128-double row), DEPTH slabs ahead
    // of the matrix cores; only the slab about to be read is waited for.
    double (*Lr)[BKD][LDP] = reinterpret_cast<double (*)[BKD][LDP]>(&Ls[0][0][0]);
    double (*Rr)[BKD][LDP] = reinterpret_cast<double (*)[BKD][LDP]>(&Rs[0][0][0]);
    // Everything but the lane offset of a direct load is wave-uniform: the LDS
    // destinations and row addresses are formed in scalar registers (a per-lane
    // address computation followed by a read-back to a scalar register cost
    // about 3% of the kernel's time).
    const int wave_u = __builtin_amdgcn_readfirstlane(wave);
    const uint32_t lds_l = __builtin_amdgcn_readfirstlane(
        (uint32_t)(uintptr_t)(lds_void*)&Lr[0][0][0]);
    const uint32_t lds_r = __builtin_amdgcn_readfirstlane(
        (uint32_t)(uintptr_t)(lds_void*)&Rr[0][0][0]);
    const uint32_t lane_b = 16u * (uint32_t)lane;
    auto issue = [&](int sl) {
      const int slot = sl % NSLOT;
#pragma unroll
      for (int h = 0; h < RPW; ++h) {
        const int row = RPW * wave_u + h;
        const uint32_t off = (uint32_t)((slot * BKD + row) * LDP) * 8u;
        const size_t grow = (size_t)(kbeg + sl * BKD + row) * n;
        const char* gl = reinterpret_cast<const char*>(L + grow + i0);
        const char* gr_ = reinterpret_cast<const char*>(R + grow + j0);
        __builtin_amdgcn_global_load_lds((const void*)(gl + lane_b),
                                         (lds_void*)(uintptr_t)(lds_l + off), 16, 0, 0);
        __builtin_amdgcn_global_load_lds((const void*)(gr_ + lane_b),
                                         (lds_void*)(uintptr_t)(lds_r + off), 16, 0, 0);
      }
    };
    const int nk = (kSplit ? ta.klen : n) / BKD;  // a multiple of FLUSHD
    // wait for slab sl: the slabs issued after it may stay in flight
    auto wait_slab = [&](int sl) {
      const int after = nk - 1 - sl;
      if (after >= 2) wait_vm<2 * LPS>();
      else if (after == 1) wait_vm<LPS>();
      else wait_vm<0>();
    };
    auto fload = [&](int slot, int kk, double* a_, double* b_) {
#pragma unroll
      for (int a = 0; a < FM; ++a) a_[a] = Lr[slot][kk + fr][wm0 + a * 16 + fc];
#pragma unroll
      for (int b = 0; b < FN; ++b) b_[b] = Rr[slot][kk + fr][wn0 + b * 16 + fc];
    };
    double av[2][FM], bv[2][FN];
    for (int d = 0; d < DEPTH && d < nk; ++d) issue(d);
    wait_slab(0);
    wg_barrier();
    if (DEPTH < nk) issue(DEPTH);
    fload(0, 0, av[0], bv[0]);
    // The slab loop is unrolled by the 64-k chain length so that the first
    // k-step of every chain is its own code: there each block's finished
    // chain is added to the running sums and its first product starts from
    // zero (no separate pass that clears the accumulators). The barrier of
    // slab sl + 1 sits before the last k-step of slab sl: by then every wave
    // holds that step's operands, so the slot can be refilled, and the next
    // slab's first operands are read from LDS while the matrix cores work on
    // the last step (no LDS latency exposed at the slab boundary).
    for (int sg = 0; sg < nk; sg += FLUSHD) {
#pragma unroll
      for (int s4 = 0; s4 < FLUSHD; ++s4) {
        const int sl = sg + s4;
        const int slot = s4;  // (sg is a multiple of NSLOT)
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int kk = 0; kk < BKD; kk += 4) {
          const int cur = (kk >> 2) & 1;
          if (kk + 4 < BKD) {
            fload(slot, kk + 4, av[cur ^ 1], bv[cur ^ 1]);
          } else {
            // (after the last slab the same steps run on no data: the wait
            // is for every load, and the operands read are not used)
            __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0): this step's operands are in
            wait_slab(sl + 1);
            wg_barrier();  // slab sl + 1 is in LDS for every wave; this slot is free
            if (sl + 1 + DEPTH < nk) issue(sl + 1 + DEPTH);
            __builtin_amdgcn_sched_barrier(0);
            fload((s4 + 1) % NSLOT, 0, av[cur ^ 1], bv[cur ^ 1]);
          }
          if (s4 == 0 && kk == 0) {
#pragma unroll
            for (int a = 0; a < FM; ++a)
#pragma unroll
              for (int b = 0; b < FN; ++b) {
                sum[a][b] += slab[a][b];
                slab[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                    av[cur][a], bv[cur][b], (v4d){0.0, 0.0, 0.0, 0.0}, 0, 0, 0);
              }
#pragma unroll
            for (int g = 0; g < 3; ++g) {
              __builtin_amdgcn_sched_group_barrier(0x002, 4, 0);  // 4 FP64 adds
              __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // 1 MFMA
              __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // 1 LDS read
            }
#pragma unroll
            for (int g = 0; g < 5; ++g) {
              __builtin_amdgcn_sched_group_barrier(0x002, 4, 0);
              __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
            }
          } else {
#pragma unroll
            for (int a = 0; a < FM; ++a)
#pragma unroll
              for (int b = 0; b < FN; ++b)
                slab[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[cur][a], bv[cur][b],
                                                                  slab[a][b], 0, 0, 0);
            {
#pragma unroll
              for (int g = 0; g < 3; ++g) {
                __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);  // 2 MFMA
                __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // 1 LDS read
              }
              __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
            }
          }
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b) sum[a][b] += slab[a][b];
    wg_barrier();  // the ring is no longer read (the epilogue's reduction reuses LDS)
  } else {
    // Loader: 32 rows x 128 columns per operand = 2048 double2; thread t moves
    // rows (t / 64) + 8q, q = 0..3, columns 2 (t % 64) and 2 (t % 64) + 1.
    const int lrow = tid >> 6;
    const int lcol = (tid & 63) * 2;
    double2 la[NQ], ra[NQ];

    auto gload = [&](int k0) {
      if (cols_in && k0 + BK <= n) {
  #pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const size_t row = (size_t)(k0 + lrow + 8 * q) * n;
          la[q] = *reinterpret_cast<const double2*>(L + row + i0 + lcol);
          ra[q] = *reinterpret_cast<const double2*>(R + row + j0 + lcol);
        }
      } else {
  #pragma unroll
        for (int q = 0; q < NQ; ++q) {
          const int k = k0 + lrow + 8 * q;
          const size_t row = (size_t)k * n;
          const bool kin = k < n;
          la[q].x = (kin && i0 + lcol < n) ? L[row + i0 + lcol] : 0.0;
          la[q].y = (kin && i0 + lcol + 1 < n) ? L[row + i0 + lcol + 1] : 0.0;
          ra[q].x = (kin && j0 + lcol < n) ? R[row + j0 + lcol] : 0.0;
          ra[q].y = (kin && j0 + lcol + 1 < n) ? R[row + j0 + lcol + 1] : 0.0;
        }
      }
    };
    auto lstore = [&](int buf) {
  #pragma unroll
      for (int q = 0; q < NQ; ++q) {
        *reinterpret_cast<double2*>(&Ls[buf][lrow + 8 * q][lcol]) = la[q];
        *reinterpret_cast<double2*>(&Rs[buf][lrow + 8 * q][lcol]) = ra[q];
      }
    };

    const int nk = (n + BK - 1) / BK;
    gload(0);
    lstore(0);
    __syncthreads();

    for (int kt = 0; kt < nk; ++kt) {
      const int buf = kt & 1;
      if (kt + 1 < nk) gload((kt + 1) * BK);
      // operands of k-step kk + 4 are read from LDS while the matrix cores
      // work on k-step kk (an LDS read between pairs of MFMAs), so the two
      // waves of a SIMD do not both wait on LDS at the start of a step
      double av[2][FM], bv[2][FN];
      auto fload = [&](int kk, double* a_, double* b_) {
  #pragma unroll
        for (int a = 0; a < FM; ++a) a_[a] = Ls[buf][kk + fr][wm0 + a * 16 + fc];
  #pragma unroll
        for (int b = 0; b < FN; ++b) b_[b] = Rs[buf][kk + fr][wn0 + b * 16 + fc];
      };
      fload(0, av[0], bv[0]);
      __builtin_amdgcn_sched_barrier(0);
  #pragma unroll
      for (int kk = 0; kk < BK; kk += 4) {
        const int cur = (kk >> 2) & 1;
        if (kk + 4 < BK) fload(kk + 4, av[cur ^ 1], bv[cur ^ 1]);
  #pragma unroll
        for (int a = 0; a < FM; ++a)
  #pragma unroll
          for (int b = 0; b < FN; ++b)
            slab[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[cur][a], bv[cur][b], slab[a][b],
                                                              0, 0, 0);
        if (kk + 4 < BK) {
  #pragma unroll
          for (int g = 0; g < 3; ++g) {
            __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);  // 2 MFMA
            __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);  // 1 LDS read
          }
          __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);
        }
        __builtin_amdgcn_sched_barrier(0);
      }
      if (kt % FLUSH == FLUSH - 1 || kt + 1 == nk) {
  #pragma unroll
        for (int a = 0; a < FM; ++a)
  #pragma unroll
          for (int b = 0; b < FN; ++b) {
            sum[a][b] += slab[a][b];
            slab[a][b] = (v4d){0.0, 0.0, 0.0, 0.0};
          }
      }
      if (kt + 1 < nk) lstore(buf ^ 1);
      __syncthreads();
    }
  }

  // Output element r of block (a, b) in this lane (the f64 16x16x4 layout,
  // checked on gfx950): row lane / 16 + 4 r, column lane % 16.
  if constexpr (kSplit) {
    const int slot = (blockIdx.x & 7) * ta.tailq + (blockIdx.x >> 3) % ta.tailq;
    double* out = ta.part + ((size_t)slot * ta.kparts + kp) * (BM * BM);
#pragma unroll
    for (int a = 0; a < FM; ++a)
#pragma unroll
      for (int b = 0; b < FN; ++b)
#pragma unroll
        for (int r = 0; r < 4; ++r)
          out[(wm0 + a * 16 + fr + 4 * r) * BM + wn0 + b * 16 + fc] = sum[a][b][r];
    return;
  }
  // Epilogue.
  double psum = 0.0;
#pragma unroll
  for (int a = 0; a < FM; ++a)
#pragma unroll
    for (int b = 0; b < FN; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        epilogue_element(e, n, tri, i0 + wm0 + a * 16 + fr + 4 * r, j0 + wn0 + b * 16 + fc,
                         sum[a][b][r], psum);
  if (e.partial) store_partial(e.partial, lw, psum, red);
}

// The split tail's tiles: the kparts range sums added in a fixed order, then
// the epilogue and the tile's partial sum. One workgroup per tile slot.
constexpr int NTR = 256;
__global__ __launch_bounds__(NTR) void tail_reduce_kernel(int n, Grid gr, int tri, Epilogue e,
                                                          TailArgs ta) {
  __shared__ double red[NTR / 64];
  const int slot = blockIdx.x;
  const int lw = (slot / ta.tailq) * ta.q + ta.qmain + slot % ta.tailq;
  int bi, bj;
  if (!(lw < gr.nreal && tri_tile_of(lw, gr, &bi, &bj))) {
    if (e.partial && threadIdx.x == 0) e.partial[lw] = 0.0;
    return;
  }
  const double* p = ta.part + (size_t)slot * ta.kparts * (BM * BM);
  double psum = 0.0;
  for (int idx = threadIdx.x; idx < BM * BM; idx += NTR) {
    double v = 0.0;
    for (int k = 0; k < ta.kparts; ++k) v += p[(size_t)k * (BM * BM) + idx];
    epilogue_element(e, n, tri, bi * BM + idx / BM, bj * BM + idx % BM, v, psum);
  }
  if (e.partial) store_partial(e.partial, lw, psum, red);
}

int launch_wgs(const Grid& gr, int tri) { return tri ? (gr.nreal + 7) / 8 * 8 : gr.nwg; }

}  // namespace

int gemm_partial_slots(int n, int tri) { return launch_wgs(make_grid(n, tri, BM), tri); }

size_t gemm_tail_scratch_elems(int n) {
  // 8 XCDs x at most 32 CUs' worth of split tiles (tailq kparts <= CUs per XCD)
  return n >= 2048 && n % BM == 0 ? (size_t)8 * 32 * BM * BM : 0;
}

hipError_t gemm_f64(const double* L, const double* R, int n, int tri, const Epilogue& e,
                    hipStream_t stream, double* scratch, size_t scratch_elems) {
  if (n <= 0) return hipSuccess;
  if (!L || !R) return hipErrorInvalidValue;  // never launch on a missing operand
  Grid gr = make_grid(n, tri, BM);
  if (tri && scratch && n % BM == 0) {
    static thread_local int ncu = 0;
    if (!ncu) {
      int dev = 0;
      if (hipGetDevice(&dev) != hipSuccess ||
          hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        ncu = 256;
    }
    const int cus = ncu / 8 > 0 ? ncu / 8 : 1;   // CUs per XCD
    const int q = (gr.nreal + 7) / 8;
    const int tailq = q % cus, qmain = q - tailq;
    if (tailq > 0 && qmain > 0) {
      int kp = cus / tailq < 4 ? cus / tailq : 4;
      while (kp > 1 && (n % (kp * 64) != 0 || (size_t)8 * tailq * kp * BM * BM > scratch_elems))
        --kp;
      if (kp > 1) {
        const TailArgs ta{q, qmain, tailq, kp, n / kp, scratch};
        hipLaunchKernelGGL(gemm_f64_kernel<false>, dim3(8 * qmain), dim3(NT), 0, stream, L, R, n,
                           gr, tri, e, ta);
        hipLaunchKernelGGL(gemm_f64_kernel<true>, dim3(8 * tailq * kp), dim3(NT), 0, stream, L, R,
                           n, gr, tri, e, ta);
        hipLaunchKernelGGL(tail_reduce_kernel, dim3(8 * tailq), dim3(NTR), 0, stream, n, gr, tri, e,
                           ta);
        return hipGetLastError();
      }
    }
  }
  hipLaunchKernelGGL(gemm_f64_kernel<false>, dim3(launch_wgs(gr, tri)), dim3(NT), 0, stream, L, R,
                     n, gr, tri, e, TailArgs{});
  return hipGetLastError();
}

}  // namespace ipr
