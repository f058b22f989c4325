// FP64 GEMM on the CDNA4 matrix cores (v_mfma_f64_16x16x4f64), LDS-staged.
//
// Workgroup = 4 waves of 64 lanes in a 2x2 arrangement; a BM x BN output tile
// per workgroup, BK = 16 per K step, double-buffered LDS, one barrier per K
// step.  Operand tiles are stored in LDS as [k][m] / [k][n] rows padded so
// that the 16-lane groups of a 64-bit LDS read fall in disjoint bank halves.
// Ragged M, N, K edges are zero-filled on load and masked on store.
#include "kernels.h"
#include "tiles.h"

namespace dcsd {

typedef double dbl4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int BK = 16;
constexpr int NT = 256;

struct KArgs {
  int64_t M, N, K;
  const double* A;
  int64_t lda;
  const double* B;
  int64_t ldb;
  double* C;
  int64_t ldc;
  double alpha, beta;
  int64_t sA, sB, sC;
  int64_t kchunk;      // K range per split (multiple of BK)
  int64_t tiles_n;
  int64_t split_stride;  // element stride between split partial outputs
  int64_t vu, nq;        // pair-blocked output (EPI = 1)
  int64_t skip_lower;    // EPI = 1, diagonal batch: skip tiles whose pairs all have p > q
  int64_t xcd_split;     // split product on a one-dimensional grid, K chunks grouped per XCD
  const double* bseg[3]; // EPI = 2: row k of B is row k % segk of bseg[k / segk]
  int64_t segk;
};

template <int BM, int BN, bool A_MC, bool B_NC, bool C_NC, bool SPLIT, int EPI = 0>
__global__ __launch_bounds__(NT) void gemm_kernel(KArgs g) {
  // LDS layouts: an operand whose M (N) index is contiguous in memory is kept
  // as [k][m] rows padded by 16 doubles (the 16-lane groups of an MFMA
  // fragment read fall in disjoint bank halves); an operand whose K index is
  // contiguous is kept as [m][k] rows of BK+1 doubles (odd stride: both the
  // row-wise stores and the fragment reads are free of bank conflicts).
  constexpr int PAD = 16;
  constexpr int LDA_S = A_MC ? BM + PAD : BK + 1;
  constexpr int LDB_S = B_NC ? BN + PAD : BK + 1;
  constexpr int SA = A_MC ? BK * LDA_S : BM * LDA_S;
  constexpr int SB = B_NC ? BK * LDB_S : BN * LDB_S;
  constexpr int LA = BM * BK / NT;
  constexpr int LB = BN * BK / NT;
  constexpr int WM = BM / 2, WN = BN / 2;
  constexpr int TM = WM / 16, TN = WN / 16;
  __shared__ double sA[2][SA];
  __shared__ double sB[2][SB];

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  int64_t tm, tn;
  if (EPI == 1 && g.skip_lower) {
    if (!diag_tile(blockIdx.x, (g.M + BM - 1) / BM, g.tiles_n, g.N, g.vu, BM, BN, tm, tn))
      return;  // whole workgroup, before any barrier
  } else {
    tile_of(blockIdx.x, (g.M + BM - 1) / BM, g.tiles_n, tm, tn);
  }
  const int64_t m0 = tm * BM, n0 = tn * BN;
  const int64_t batch = blockIdx.y;
  const double* A = g.A + batch * g.sA;
  const double* B = g.B + batch * g.sB;

  int64_t kbeg = 0, kend = g.K;
  if (SPLIT) {
    kbeg = (int64_t)blockIdx.z * g.kchunk;
    kend = kbeg + g.kchunk < g.K ? kbeg + g.kchunk : g.K;
  }

  // Element e = tid + i*NT of a K step sits at a thread part (fixed over the K loop and
  // kept as a 32-bit byte offset) plus a part that only depends on i: the load address
  // is a uniform base plus the thread's offset, so no per-element 64-bit address lives
  // in registers across the loop (the host bounds the offsets below 2^32 bytes).
  const int ka0 = A_MC ? tid / BM : tid % BK, ma0 = A_MC ? tid % BM : tid / BK;
  const int kb0 = B_NC ? tid / BN : tid % BK, nb0 = B_NC ? tid % BN : tid / BK;
  constexpr int AK = A_MC ? NT / BM : 0, AM = A_MC ? 0 : NT / BK;  // per-i steps of (k, m)
  constexpr int BKS = B_NC ? NT / BN : 0, BNS = B_NC ? 0 : NT / BK;
  const uint32_t aoff = (uint32_t)(8 * (A_MC ? ma0 + ka0 * g.lda : ma0 * g.lda + ka0));
  const uint32_t boff = (uint32_t)(8 * (B_NC ? nb0 + kb0 * g.ldb : nb0 * g.ldb + kb0));
  double ra[LA], rb[LB];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int i = 0; i < LA; ++i) {
      const int64_t gm = m0 + ma0 + i * AM, gk = k0 + ka0 + i * AK;
      const double* base = A + (A_MC ? (m0 + i * AM) + (k0 + i * AK) * g.lda : (m0 + i * AM) * g.lda + k0 + i * AK);
      ra[i] = (gm < g.M && gk < kend) ? *(const double*)((const char*)base + aoff) : 0.0;
    }
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      const int64_t gn = n0 + nb0 + i * BNS, gk = k0 + kb0 + i * BKS;
      const double* base = B + (B_NC ? (n0 + i * BNS) + (k0 + i * BKS) * g.ldb : (n0 + i * BNS) * g.ldb + k0 + i * BKS);
      rb[i] = (gn < g.N && gk < kend) ? *(const double*)((const char*)base + boff) : 0.0;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int i = 0; i < LA; ++i) {
      const int e = tid + i * NT;
      int k, m;
      if (A_MC) { k = e / BM; m = e % BM; } else { k = e % BK; m = e / BK; }
      sA[buf][A_MC ? k * LDA_S + m : m * LDA_S + k] = ra[i];
    }
#pragma unroll
    for (int i = 0; i < LB; ++i) {
      const int e = tid + i * NT;
      int k, n;
      if (B_NC) { k = e / BN; n = e % BN; } else { k = e % BK; n = e / BK; }
      sB[buf][B_NC ? k * LDB_S + n : n * LDB_S + k] = rb[i];
    }
  };

  dbl4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};

  const int64_t nk = (kend - kbeg + BK - 1) / BK;
  if (nk > 0) {
    load(kbeg);
    store(0);
  }
  __syncthreads();
  const int lrow = lane >> 4, lcol = lane & 15;
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int buf = (int)(kt & 1);
    if (kt + 1 < nk) load(kbeg + (kt + 1) * BK);
    const double* a_s = sA[buf];
    const double* b_s = sB[buf];
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      double af[TM], bf[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int mm = wm * WM + i * 16 + lcol, kk = ks * 4 + lrow;
        af[i] = a_s[A_MC ? kk * LDA_S + mm : mm * LDA_S + kk];
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int nn = wn * WN + j * 16 + lcol, kk = ks * 4 + lrow;
        bf[j] = b_s[B_NC ? kk * LDB_S + nn : nn * LDB_S + kk];
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
    if (kt + 1 < nk) store(buf ^ 1);
    __syncthreads();
  }

  // epilogue: for the FP64 16x16x4 MFMA, lane holds D[lane/16 + 4*r][lane%16] of each 16x16 tile
  double* C = g.C + batch * g.sC;
  if (SPLIT) C += (int64_t)blockIdx.z * g.split_stride;
  const int64_t mb = m0 + wm * WM + lrow, nbase = n0 + wn * WN + lcol;
  if constexpr (EPI == 1) {
    // m = (p, c), n = (q, d) -> V2[(p*nq + q)][c][d]: the offset splits into a row part
    // p*nq*vu^2 + c*vu and a column part q*vu^2 + d, both stepped without divisions
    const int vu = (int)g.vu;
    const int64_t vv = g.vu * g.vu;
    int64_t coff[TN];
    {
      int q = (int)(nbase / vu), d = (int)(nbase % vu);
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        coff[j] = (int64_t)q * vv + d;
        d += 16;
        while (d >= vu) {
          d -= vu;
          ++q;
        }
      }
    }
    int p = (int)(mb / vu), c = (int)(mb % vu);
#pragma unroll
    for (int i = 0; i < TM; ++i) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (mb + i * 16 + 4 * r < g.M) {
          const int64_t roff = (int64_t)p * g.nq * vv + (int64_t)c * vu;
#pragma unroll
          for (int j = 0; j < TN; ++j)
            if (nbase + j * 16 < g.N) C[roff + coff[j]] = acc[i][j][r];
        }
        c += 4;
        while (c >= vu) {
          c -= vu;
          ++p;
        }
      }
    }
    return;
  }
  if constexpr (SPLIT) {
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int j = 0; j < TN; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int64_t gm = mb + i * 16 + 4 * r;
          const int64_t gn = nbase + j * 16;
          if (gm < g.M && gn < g.N) C[C_NC ? gm * g.ldc + gn : gm + gn * g.ldc] = acc[i][j][r];
        }
    return;
  }
  // alpha/beta epilogue staged through LDS, one 16-row block of the wave tile at a
  // time: the accumulators go to LDS straight from the matrix-core registers (scaling
  // them in place would copy all of them to VGPRs, inside the K loop as well), and the
  // C reads and writes become contiguous along C's leading dimension
  constexpr int SROW = WN + 1;
  static_assert(4 * 16 * SROW <= 2 * SA, "epilogue staging does not fit");
  double* stg = &sA[0][0] + wave * 16 * SROW;
  const int64_t mw = m0 + wm * WM, nw = n0 + wn * WN;
#pragma unroll
  for (int i = 0; i < TM; ++i) {
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) stg[(lrow + 4 * r) * SROW + j * 16 + lcol] = acc[i][j][r];
    __syncthreads();
#pragma unroll
    for (int t = 0; t < 16 * WN / 64; ++t) {
      const int e = lane + 64 * t;
      const int rr = C_NC ? e / WN : e % 16, cc = C_NC ? e % WN : e / 16;
      const int64_t gm = mw + i * 16 + rr, gn = nw + cc;
      if (gm < g.M && gn < g.N) {
        const int64_t off = C_NC ? gm * g.ldc + gn : gm + gn * g.ldc;
        double v = g.alpha * stg[rr * SROW + cc];
        if (g.beta != 0.0) v += g.beta * C[off];
        C[off] = v;
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// Direct-to-LDS GEMM.  Each K step's operand tiles go from global memory
// straight into LDS (global_load_lds_dwordx4: 16 bytes per lane, 1 KiB per wave
// instruction) through a ring of S LDS stages with BK = 8, on 8 waves holding
// 4 x 2 wave tiles of 32 x 64 (four waves per SIMD).  A step waits until its own
// stage has landed (S - 2 younger steps stay in flight), reads all of its
// fragments, issues the step S - 1 ahead into the stage read one step earlier,
// then runs its MFMAs, so the loads overlap S - 1 steps of matrix work without
// register staging.  The fragment reads are written as LDS reads that wait for
// their own results inside the same asm block, and the step barrier is a bare
// s_barrier: the compiler's own waits before LDS reads and at workgroup fences
// would drain every load in flight, including the younger stages.
//
// Operand layouts (KM = true: the operand's M (N) index is contiguous, stored
// [k][m]; KM = false: its K index is contiguous, stored [m][k]):
//  * KM tile: 8 rows (k) of 128 doubles, padded to DL_ROW; wave w loads row w.
//  * K-contiguous tile: 128 rows (m) of 8 doubles; wave w loads rows 16w..16w+15,
//    4 lanes per row, and each lane fetches the 16-byte chunk that lands in its
//    slot under the swizzle slot = chunk ^ ((row >> 2) & 3), which spreads the
//    16 rows of an MFMA fragment read over distinct LDS banks.
// Lanes whose elements lie past M (N) or past the K range read a zero row.
// Needs even extents along each operand's contiguous index, even leading
// dimensions and batch strides, and 16-byte aligned A, B.
constexpr int DL_BK = 8, DL_WGM = 4, DL_WGN = 2, DL_NW = DL_WGM * DL_WGN, DL_NT = 64 * DL_NW;
constexpr int DL_ROW = 128 + 16;
__device__ __attribute__((aligned(16))) double dl_zero_row[128];

template <bool KM>
struct DlTile {
  static constexpr int SIZE = KM ? DL_BK * DL_ROW : 128 * DL_BK;  // doubles per stage
  // LDS index of element (r, k) of the tile (r: row along M or N within the tile)
  static __device__ int at(int r, int k) {
    return KM ? k * DL_ROW + r : r * DL_BK + 2 * ((k >> 1) ^ ((r >> 2) & 3)) + (k & 1);
  }
  // this lane's global source for the wave's share of the step starting at k0
  static __device__ const double* src(const double* P, int64_t ld, int64_t o0, int64_t extent, int64_t k0,
                                      int64_t kend, int wave, int lane, const double* zrow) {
    if (KM) {
      const int64_t k = k0 + wave;
      return (o0 + 2 * lane < extent && k < kend) ? P + k * ld + o0 + 2 * lane : zrow;
    }
    const int r = wave * 16 + (lane >> 2);
    const int chunk = (lane & 3) ^ ((r >> 2) & 3);
    const int64_t k = k0 + 2 * chunk;
    return (o0 + r < extent && k < kend) ? P + (o0 + r) * ld + k : zrow;
  }
  static __device__ int dst(int wave) { return KM ? wave * DL_ROW : wave * 128; }
};

__device__ inline uint32_t lds_byte_address(const void* p) {
  return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void*)p;
}

// s_waitcnt immediate: at most `vm` vector-memory operations outstanding, no other wait
constexpr int waitcnt_vm(int vm) { return (vm & 0xF) | ((vm >> 4) << 14) | (7 << 4) | (0xF << 8); }

template <bool A_KM, bool B_KM, int EPI, bool SPLIT, bool C_NC>
__global__ __launch_bounds__(DL_NT) void gemm_dl_kernel(KArgs g) {
  static_assert(EPI != 2 || (B_KM && !SPLIT), "segmented B: K-major, whole K");
  constexpr int BM = 128, BN = 128;
  constexpr int WM = BM / DL_WGM, WN = BN / DL_WGN, TM = WM / 16, TN = WN / 16, KS = DL_BK / 4;
  static_assert(DL_NW == DL_BK && DL_NW * 16 == BM, "one wave instruction per operand per step");
  static_assert(TM == 2 && TN == 4 && KS == 2, "the fragment reads below are written for 2 x 4 fragments");
  // K-major tiles stream from L2 (two stages suffice); K-contiguous ones see longer latency
  constexpr int S = (A_KM && B_KM) ? 2 : 4;
  using TA = DlTile<A_KM>;
  using TB = DlTile<B_KM>;
  __shared__ __attribute__((aligned(16))) double sA[S][TA::SIZE];
  __shared__ __attribute__((aligned(16))) double sB[S][TB::SIZE];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / DL_WGN, wn = wave % DL_WGN;
  int64_t tm, tn;
  int64_t z = blockIdx.z;
  if (EPI == 1 && g.skip_lower) {
    if (!diag_tile(blockIdx.x, (g.M + BM - 1) / BM, g.tiles_n, g.N, g.vu, BM, BN, tm, tn))
      return;  // whole workgroup, before any barrier
  } else if (SPLIT && g.xcd_split) {
    // one matrix, K chunks grouped per XCD: the chunk's A rows and B columns are fetched once
    // into one L2 instead of once per XCD that holds one of its tiles
    z = split_tile_of(blockIdx.x, (g.M + BM - 1) / BM, g.tiles_n, tm, tn);
  } else {
    tile_of(blockIdx.x, (g.M + BM - 1) / BM, g.tiles_n, tm, tn);
  }
  const int64_t m0 = tm * BM, n0 = tn * BN;
  const int64_t batch = blockIdx.y;
  int64_t kbeg = 0, kend = g.K;
  if (SPLIT) {
    kbeg = z * g.kchunk;
    kend = kbeg + g.kchunk < g.K ? kbeg + g.kchunk : g.K;
  }
  const double* zrow = dl_zero_row + 2 * lane;
  const double* A = g.A + batch * g.sA;
  const double* B = g.B + batch * g.sB;
  auto issue = [&](int slot, int64_t k0) {
    const double* sa = TA::src(A, g.lda, m0, g.M, k0, kend, wave, lane, zrow);
    const double* sb;
    if constexpr (EPI == 2) {
      // K-major B in segments: this wave's row k lies in segment k / segk (wave-uniform)
      const int64_t k = k0 + wave;
      sb = zrow;
      if (n0 + 2 * lane < g.N && k < kend) {
        const int64_t q = k / g.segk;
        sb = g.bseg[q] + (k - q * g.segk) * g.ldb + n0 + 2 * lane;
      }
    } else {
      sb = TB::src(B, g.ldb, n0, g.N, k0, kend, wave, lane, zrow);
    }
    __builtin_amdgcn_global_load_lds((const void*)sa, (void __attribute__((address_space(3)))*)&sA[slot][TA::dst(wave)],
                                     16, 0, 0);
    __builtin_amdgcn_global_load_lds((const void*)sb, (void __attribute__((address_space(3)))*)&sB[slot][TB::dst(wave)],
                                     16, 0, 0);
  };

  dbl4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = dbl4{0.0, 0.0, 0.0, 0.0};
  const int lrow = lane >> 4, lcol = lane & 15;
  // byte offsets of this lane's fragments within a stage, per k sub-step; the next
  // 16 rows of a tile sit a fixed distance further in both layouts
  uint32_t ao[KS], bo[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    ao[ks] = 8u * (uint32_t)TA::at(wm * WM + lcol, ks * 4 + lrow);
    bo[ks] = 8u * (uint32_t)TB::at(wn * WN + lcol, ks * 4 + lrow);
  }
  constexpr uint32_t AI = 8u * (A_KM ? 16 : 16 * DL_BK), BJ = 8u * (B_KM ? 16 : 16 * DL_BK);
  const int64_t nk = (kend - kbeg + DL_BK - 1) / DL_BK;
#pragma unroll
  for (int t = 0; t < S - 1; ++t) issue(t, kbeg + t * DL_BK);
  for (int64_t kt = 0; kt < nk; ++kt) {
    // this wave's loads of step kt have landed (the S - 2 younger steps may not have);
    // after the barrier everyone's have, and every wave has finished reading the stage
    // that the issue below refills (it was read at step kt - 1)
    __builtin_amdgcn_s_waitcnt(waitcnt_vm(2 * (S - 2)));
    __builtin_amdgcn_s_barrier();
    const int slot = (int)(kt & (S - 1));
    const uint32_t sa = lds_byte_address(sA[slot]), sb = lds_byte_address(sB[slot]);
    // each k sub-step's fragments are read just before its MFMAs, so that a wave's
    // second read overlaps the MFMAs it has already issued; B fragments 2-3 are read after
    // the MFMAs of fragments 0-1 are issued (each accumulator's MFMA order is unchanged)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      double af[TM], bf[TN];
      const uint32_t pa = sa + ao[ks], pb = sb + bo[ks];
      asm volatile(
          "ds_read_b64 %0, %4\n"
          "ds_read_b64 %1, %4 offset:%6\n"
          "ds_read_b64 %2, %5\n"
          "ds_read_b64 %3, %5 offset:%7\n"
          "s_waitcnt lgkmcnt(0)"
          : "=&v"(af[0]), "=&v"(af[1]), "=&v"(bf[0]), "=&v"(bf[1])
          : "v"(pa), "v"(pb), "n"(AI), "n"(BJ)
          : "memory");
      if (ks == 0) issue((int)((kt + S - 1) & (S - 1)), kbeg + (kt + S - 1) * DL_BK);  // past kend: zero rows
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
      asm volatile(
          "ds_read_b64 %0, %2 offset:%3\n"
          "ds_read_b64 %1, %2 offset:%4\n"
          "s_waitcnt lgkmcnt(0)"
          : "=&v"(bf[2]), "=&v"(bf[3])
          : "v"(pb), "n"(2 * BJ), "n"(3 * BJ)
          : "memory");
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 2; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
  }
  __builtin_amdgcn_s_waitcnt(0);  // the last (zero) stage has landed before the wave retires

  double* C = g.C + batch * g.sC;
  if (SPLIT) C += z * g.split_stride;
  const int64_t mb = m0 + wm * WM + lrow, nbase = n0 + wn * WN + lcol;
  if constexpr (EPI == 1) {
    // m = (p, c), n = (q, d) -> V2[(p*nq + q)][c][d], offsets stepped as in gemm_kernel
    const int vu = (int)g.vu;
    const int64_t vv = g.vu * g.vu;
    int64_t coff[TN];
    {
      int q = (int)(nbase / vu), d = (int)(nbase % vu);
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        coff[j] = (int64_t)q * vv + d;
        d += 16;
        while (d >= vu) {
          d -= vu;
          ++q;
        }
      }
    }
    int p = (int)(mb / vu), c = (int)(mb % vu);
#pragma unroll
    for (int i = 0; i < TM; ++i) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (mb + i * 16 + 4 * r < g.M) {
          const int64_t roff = (int64_t)p * g.nq * vv + (int64_t)c * vu;
#pragma unroll
          for (int j = 0; j < TN; ++j)
            if (nbase + j * 16 < g.N) C[roff + coff[j]] = acc[i][j][r];
        }
        c += 4;
        while (c >= vu) {
          c -= vu;
          ++p;
        }
      }
    }
    return;
  }
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gm = mb + i * 16 + 4 * r, gn = nbase + j * 16;
        if (gm < g.M && gn < g.N) {
          const int64_t off = C_NC ? gm * g.ldc + gn : gm + gn * g.ldc;
          if (SPLIT) {
            C[off] = acc[i][j][r];
          } else {
            double v = g.alpha * acc[i][j][r];
            if (g.beta != 0.0) v += g.beta * C[off];
            C[off] = v;
          }
        }
      }
}

// The direct-to-LDS kernel streams each operand row in 16-byte chunks along its contiguous
// extent (K for a K-contiguous operand, M or N for a K-major one): every row must start
// 16-byte aligned (even leading dimension and batch stride, aligned base) and an odd extent
// needs an element past its end that is zero, which the padded copy below provides.
bool operand_ok(const double* p, int64_t ld, int64_t extent, int64_t stride, int64_t batch) {
  return extent % 2 == 0 && ld % 2 == 0 && ((uintptr_t)p & 15) == 0 && (batch == 1 || stride % 2 == 0);
}
bool dl_ok(const GemmArgs& g) {
  return operand_ok(g.A, g.lda, g.a_mc ? g.M : g.K, g.sA, g.batch) &&
         operand_ok(g.B, g.ldb, g.b_nc ? g.N : g.K, g.sB, g.batch);
}
// whether the output has the tiles the direct-to-LDS kernel takes
bool dl_shape(const GemmArgs& g) {
  const int64_t tiles128 = ((g.M + 127) / 128) * ((g.N + 127) / 128) * g.batch * g.ksplit;
  return g.M >= 128 && g.N >= 128 && tiles128 >= 128;
}

// Zero-padded copy of an operand: `rows` rows of `extent` contiguous elements (leading
// dimension ld, batch stride stride; stride 0: one matrix shared by the batch) into rows of
// ldp = extent rounded up to even, the batch's matrices back to back.
struct PadPlan {
  bool copy = false;
  int64_t rows = 0, extent = 0, ldp = 0, nb = 0;
  int64_t elems() const { return copy ? (nb * rows * ldp + 1) / 2 * 2 : 0; }  // keeps what follows aligned
  int64_t stride() const { return nb > 1 ? rows * ldp : 0; }
};
PadPlan pad_plan(const double* p, int64_t ld, int64_t extent, int64_t rows, int64_t stride, int64_t batch) {
  PadPlan q;
  if (operand_ok(p, ld, extent, stride, batch)) return q;
  q.copy = true;
  q.rows = rows;
  q.extent = extent;
  q.ldp = extent + (extent & 1);
  q.nb = batch > 1 && stride != 0 ? batch : 1;
  return q;
}
PadPlan pad_plan_a(const GemmArgs& g) {
  return pad_plan(g.A, g.lda, g.a_mc ? g.M : g.K, g.a_mc ? g.K : g.M, g.sA, g.batch);
}
PadPlan pad_plan_b(const GemmArgs& g) {
  return pad_plan(g.B, g.ldb, g.b_nc ? g.N : g.K, g.b_nc ? g.K : g.N, g.sB, g.batch);
}

// dst[(b * rows + r) * ldp + c] = c < extent ? src[b * stride + r * ld + c] : 0
__global__ __launch_bounds__(256) void pad_copy_kernel(double* dst, int64_t ldp, const double* src, int64_t ld,
                                                      int64_t stride, int64_t rows, int64_t extent, int64_t total) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = i / ldp, c = i - row * ldp, b = row / rows, r = row - b * rows;
    dst[i] = c < extent ? src[b * stride + r * ld + c] : 0.0;
  }
}

void pad_copy(const PadPlan& q, double* dst, const double* src, int64_t ld, int64_t stride, hipStream_t s) {
  const int64_t total = q.nb * q.rows * q.ldp;
  int64_t blocks = (total + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(pad_copy_kernel, dim3((unsigned)blocks), dim3(256), 0, s, dst, q.ldp, src, ld, stride, q.rows,
                     q.extent, total);
  DCSD_CHECK_LAUNCH();
}

template <bool A_KM, bool B_KM, bool C_NC>
void launch_dl3(const GemmArgs& g, KArgs& k, hipStream_t s) {
  const int64_t tm = (g.M + 127) / 128, tn = (g.N + 127) / 128;
  k.tiles_n = tn;
  dim3 grid((unsigned)(tm * tn), (unsigned)g.batch, (unsigned)g.ksplit);
  k.xcd_split = g.ksplit > 1 && g.ksplit % 8 == 0 && g.batch == 1 ? 1 : 0;
  if (k.xcd_split) grid = dim3((unsigned)(tm * tn * g.ksplit));
  if (g.ksplit > 1)
    hipLaunchKernelGGL((gemm_dl_kernel<A_KM, B_KM, 0, true, C_NC>), grid, dim3(DL_NT), 0, s, k);
  else
    hipLaunchKernelGGL((gemm_dl_kernel<A_KM, B_KM, 0, false, C_NC>), grid, dim3(DL_NT), 0, s, k);
}

void launch_dl(const GemmArgs& g, KArgs& k, hipStream_t s) {
  const int code = (g.a_mc ? 4 : 0) | (g.b_nc ? 2 : 0) | (g.c_nc ? 1 : 0);
  switch (code) {
    case 0: launch_dl3<false, false, false>(g, k, s); break;
    case 1: launch_dl3<false, false, true>(g, k, s); break;
    case 2: launch_dl3<false, true, false>(g, k, s); break;
    case 3: launch_dl3<false, true, true>(g, k, s); break;
    case 4: launch_dl3<true, false, false>(g, k, s); break;
    case 5: launch_dl3<true, false, true>(g, k, s); break;
    case 6: launch_dl3<true, true, false>(g, k, s); break;
    default: launch_dl3<true, true, true>(g, k, s); break;
  }
}

// C = alpha * sum_z W[z] + beta * C, W[z] laid out like C (same ldc/c_nc/batch strides).
__global__ void split_reduce(const double* W, double* C, int64_t M, int64_t N, int64_t ldc, bool c_nc,
                             int64_t batch, int64_t sC, int nsplit, int64_t split_stride, double alpha,
                             double beta) {
  const int64_t total = M * N * batch;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = idx / (M * N);
    const int64_t r = idx % (M * N);
    const int64_t m = c_nc ? r / N : r % M;
    const int64_t n = c_nc ? r % N : r / M;
    const int64_t off = b * sC + (c_nc ? m * ldc + n : m + n * ldc);
    double s = 0.0;
    for (int z = 0; z < nsplit; ++z) s += W[z * split_stride + off];
    double v = alpha * s;
    if (beta != 0.0) v += beta * C[off];
    C[off] = v;
  }
}

template <int BM, int BN, bool A_MC, bool B_NC, bool C_NC>
void launch(const GemmArgs& g, KArgs& k, hipStream_t s) {
  const int64_t tm = (g.M + BM - 1) / BM, tn = (g.N + BN - 1) / BN;
  k.tiles_n = tn;
  dim3 grid((unsigned)(tm * tn), (unsigned)g.batch, (unsigned)g.ksplit);
  if (g.ksplit > 1)
    hipLaunchKernelGGL((gemm_kernel<BM, BN, A_MC, B_NC, C_NC, true>), grid, dim3(NT), 0, s, k);
  else
    hipLaunchKernelGGL((gemm_kernel<BM, BN, A_MC, B_NC, C_NC, false>), grid, dim3(NT), 0, s, k);
}

template <int BM, int BN>
void dispatch(const GemmArgs& g, KArgs& k, hipStream_t s) {
  const int code = (g.a_mc ? 4 : 0) | (g.b_nc ? 2 : 0) | (g.c_nc ? 1 : 0);
  switch (code) {
    case 0: launch<BM, BN, false, false, false>(g, k, s); break;
    case 1: launch<BM, BN, false, false, true>(g, k, s); break;
    case 2: launch<BM, BN, false, true, false>(g, k, s); break;
    case 3: launch<BM, BN, false, true, true>(g, k, s); break;
    case 4: launch<BM, BN, true, false, false>(g, k, s); break;
    case 5: launch<BM, BN, true, false, true>(g, k, s); break;
    case 6: launch<BM, BN, true, true, false>(g, k, s); break;
    default: launch<BM, BN, true, true, true>(g, k, s); break;
  }
}

}  // namespace

// Padding pays where the copies are small against the product: at least 256 flops per
// copied element (for a single operand, the other operand's extent of 128 or more).
int64_t gemm_f64_pad_work(const GemmArgs& g) {
  if (g.M <= 0 || g.N <= 0 || g.K <= 0 || g.batch <= 0 || !dl_shape(g) || dl_ok(g)) return 0;
  const PadPlan pa = pad_plan_a(g), pb = pad_plan_b(g);
  if (pa.ldp >= ((int64_t)1 << 25) || pb.ldp >= ((int64_t)1 << 25)) return 0;
  const int64_t n = pa.elems() + pb.elems();
  const double flops = 2.0 * (double)g.M * (double)g.N * (double)g.K * (double)g.batch;
  return flops >= 256.0 * (double)n ? n : 0;
}

void gemm_f64(const GemmArgs& g, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0 || g.batch <= 0) return;
  if (g.batch > 65535 || g.ksplit > 65535 || g.ksplit < 1) throw ArgError("gemm_f64: grid too large");
  // the kernels keep each thread's operand offset within a K step as 32-bit bytes
  if (g.lda >= ((int64_t)1 << 25) || g.ldb >= ((int64_t)1 << 25))
    throw ArgError("gemm_f64: leading dimension too large");
  KArgs k{};
  k.M = g.M; k.N = g.N; k.K = g.K;
  k.A = g.A; k.lda = g.lda; k.B = g.B; k.ldb = g.ldb;
  k.C = g.C; k.ldc = g.ldc; k.alpha = g.alpha; k.beta = g.beta;
  k.sA = g.sA; k.sB = g.sB; k.sC = g.sC;
  if (g.ksplit > 1) {
    if (!g.work) throw ArgError("gemm_f64: split-K needs a workspace");
    int64_t chunk = (g.K + g.ksplit - 1) / g.ksplit;
    chunk = (chunk + BK - 1) / BK * BK;
    k.kchunk = chunk;
    k.C = g.work;
    // partials use the same C addressing with sC, plus a per-split stride
    int64_t span = (g.batch - 1) * g.sC + (g.c_nc ? (g.M - 1) * g.ldc + g.N : (g.N - 1) * g.ldc + g.M);
    k.split_stride = span;
  } else {
    k.kchunk = g.K;
    k.split_stride = 0;
  }
  const int64_t pad = gemm_f64_pad_work(g);
  if (dl_shape(g) && pad > 0 && g.pad && pad <= g.pad_cap) {
    // copy the operands the direct-to-LDS kernel cannot stream into the padded workspace
    const PadPlan pa = pad_plan_a(g), pb = pad_plan_b(g);
    double* w = g.pad;
    if (pa.copy) {
      pad_copy(pa, w, g.A, g.lda, g.sA, s);
      k.A = w;
      k.lda = pa.ldp;
      k.sA = pa.stride();
      w += pa.elems();
    }
    if (pb.copy) {
      pad_copy(pb, w, g.B, g.ldb, g.sB, s);
      k.B = w;
      k.ldb = pb.ldp;
      k.sB = pb.stride();
    }
    launch_dl(g, k, s);
  } else if (dl_shape(g) && dl_ok(g)) {
    launch_dl(g, k, s);
  } else if (dl_shape(g))
    dispatch<128, 128>(g, k, s);
  else
    dispatch<64, 64>(g, k, s);
  DCSD_CHECK_LAUNCH();
  if (g.ksplit > 1) {
    const int64_t total = g.M * g.N * g.batch;
    int blocks = (int)((total + 255) / 256);
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(split_reduce, dim3(blocks), dim3(256), 0, s, (const double*)g.work, g.C, g.M, g.N,
                       g.ldc, g.c_nc, g.batch, g.sC, g.ksplit, k.split_stride, g.alpha, g.beta);
    DCSD_CHECK_LAUNCH();
  }
}

bool gemm_f64_bseg(int64_t M, int64_t N, int64_t segk, int nseg, const double* A, int64_t lda,
                   const double* const* bseg, int64_t ldb, double* C, int64_t ldc, double alpha, double beta,
                   hipStream_t s) {
  if (nseg < 1 || nseg > 3 || segk < 1 || M < 128 || N < 128) return false;
  const int64_t K = nseg * segk, tm = (M + 127) / 128, tn = (N + 127) / 128;
  const auto al16 = [](const void* p) { return ((uintptr_t)p & 15) == 0; };
  bool ok = tm * tn >= 128 && lda % 2 == 0 && lda >= K + (K & 1) && al16(A) && N % 2 == 0 && ldb % 2 == 0 &&
            lda < ((int64_t)1 << 25) && ldb < ((int64_t)1 << 25);
  for (int q = 0; q < nseg; ++q) ok = ok && bseg[q] && al16(bseg[q]);
  if (!ok) return false;
  KArgs k{};
  k.M = M; k.N = N; k.K = K;
  k.A = A; k.lda = lda;
  k.B = bseg[0]; k.ldb = ldb;
  for (int q = 0; q < 3; ++q) k.bseg[q] = bseg[q < nseg ? q : 0];
  k.segk = segk;
  k.C = C; k.ldc = ldc; k.alpha = alpha; k.beta = beta;
  k.kchunk = K;
  k.tiles_n = tn;
  hipLaunchKernelGGL((gemm_dl_kernel<false, true, 2, false, true>), dim3((unsigned)(tm * tn)), dim3(DL_NT), 0, s, k);
  DCSD_CHECK_LAUNCH();
  return true;
}

// Ladder integral batch: V2[(p*nq + q)][c][d] = sum_P Bl[P][p0+p][c] Bl[P][q0+q][d]
// with Bl laid out [P][row][c] (row stride vu, P stride ld).
void gemm_f64_pairs(const double* Bl, int64_t ld, int64_t vu, int64_t naux, int64_t p0, int64_t np, int64_t q0,
                    int64_t nq, double* V2, hipStream_t s) {
  if (ld >= ((int64_t)1 << 25)) throw ArgError("gemm_f64_pairs: leading dimension too large");
  KArgs k{};
  k.M = np * vu; k.N = nq * vu; k.K = naux;
  k.A = Bl + p0 * vu; k.lda = ld;
  k.B = Bl + q0 * vu; k.ldb = ld;
  k.C = V2; k.ldc = 0; k.alpha = 1.0; k.beta = 0.0;
  k.kchunk = naux; k.vu = vu; k.nq = nq;
  // a diagonal batch is symmetric under (p, c) <-> (q, d): the tiles entirely in p > q are
  // skipped and those pairs copied from their mirrors below
  const int64_t tm = (k.M + 127) / 128, tn = (k.N + 127) / 128;
  k.tiles_n = tn;
  k.skip_lower = p0 == q0 && np == nq && np * (np - 1) / 2 <= 65535 && diag_skips(np, vu, 128, 128);
  const int64_t grid = k.skip_lower ? diag_grid(tm, tn) : tm * tn;
  const bool al = (((uintptr_t)k.A | (uintptr_t)k.B) & 15) == 0;
  if (k.M % 2 == 0 && k.N % 2 == 0 && ld % 2 == 0 && al)
    hipLaunchKernelGGL((gemm_dl_kernel<true, true, 1, false, true>), dim3((unsigned)grid), dim3(DL_NT), 0, s, k);
  else
    hipLaunchKernelGGL((gemm_kernel<128, 128, true, true, true, false, 1>), dim3((unsigned)grid), dim3(NT), 0, s, k);
  DCSD_CHECK_LAUNCH();
  if (k.skip_lower) {
    const int tiles = (int)((vu + 31) / 32);
    hipLaunchKernelGGL(pair_mirror_kernel<double>, dim3((unsigned)(tiles * tiles), (unsigned)(np * (np - 1) / 2)), dim3(256), 0, s,
                       V2, vu, vu * vu, np, tiles);
    DCSD_CHECK_LAUNCH();
  }
}

}  // namespace dcsd
