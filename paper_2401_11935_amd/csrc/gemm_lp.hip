// Low-precision GEMMs on the CDNA4 matrix cores with FP32 accumulation:
// FP32 inputs (v_mfma_f32_16x16x4_f32) or BF16 inputs (v_mfma_f32_16x16x32_bf16).
//
// Both operands are K-contiguous in memory, A(m,k) = A[m*lda + k] and
// B(k,n) = B[n*ldb + k], with lda and ldb multiples of 8 elements and
// 16-byte aligned bases, so that every global load is one 16-byte vector and
// every LDS row stays 16-byte aligned.  Tiles of 128 x 128 per workgroup of
// four waves (2 x 2, 64 x 64 each), K staged through double-buffered LDS rows
// padded to a bank-conflict-free stride.
//
// Epilogues: FP32 split-K partials (reduced into FP64 in a fixed order), the
// pair-blocked ladder integrals V2[(p,q)][c][d] in the input precision, or a
// direct FP64 update C = alpha*AB + beta*C.
#include <hip/hip_bf16.h>
#include <algorithm>

#include "../../include/libdcsd.h"
#include "kernels.h"
#include "tiles.h"

namespace dcsd {

namespace {

typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

constexpr int NT = 256;
constexpr int TILE = 128;
__device__ __attribute__((aligned(16))) unsigned char lp_zero_row[64 * 16];  // zero source for rows past M, N, K

enum { EPI_SPLIT = 0, EPI_PAIRS = 1, EPI_F64 = 2 };

struct LArgs {
  int64_t M, N, K;
  const void* A;
  int64_t lda;
  const void* B;
  int64_t ldb;
  void* C;
  int64_t ldc;
  int c_nc;
  double alpha, beta;
  int64_t kchunk, tiles_n, split_stride;
  int64_t vu, nq, kp;  // pair-blocked output
  int64_t skip_lower;  // pair-blocked diagonal batch: skip tiles whose pairs all have p > q
  int64_t xcd_split;   // split product on a one-dimensional grid, chunks grouped per XCD
};

template <class T>
struct Traits;
template <>
struct Traits<float> {
  static constexpr int VL = 4;     // elements per 16-byte load
  static constexpr int KSTEP = 4;  // K per MFMA
};
template <>
struct Traits<__bf16> {
  static constexpr int VL = 8;
  static constexpr int KSTEP = 32;
};

// Rounding of an FP32 value to the storage precision, nearest even, written
// out so that the result does not depend on how the compiler lowers casts
// (a quiet NaN stays a NaN).
template <class T>
__device__ inline T lp_round(float x);
template <>
__device__ inline float lp_round<float>(float x) { return x; }
template <>
__device__ inline __bf16 lp_round<__bf16>(float x) {
  uint32_t b = __float_as_uint(x);
  const uint16_t h = (b & 0x7fffffffu) > 0x7f800000u ? (uint16_t)0x7fc0u
                                                      : (uint16_t)((b + 0x7fffu + ((b >> 16) & 1u)) >> 16);
  return __builtin_bit_cast(__bf16, h);
}

template <class T>
__device__ inline uint4 load_chunk(const T* p, int64_t kk, int64_t kend) {
  constexpr int VL = Traits<T>::VL;
  if (kk + VL <= kend) return *reinterpret_cast<const uint4*>(p);
  union {
    uint4 u;
    T e[VL];
  } x;
#pragma unroll
  for (int e = 0; e < VL; ++e) x.e[e] = (kk + e < kend) ? p[e] : (T)0.0f;
  return x.u;
}

// K depth of one LDS stage: 16 FP32 / 64 BF16 elements with 128-row tiles,
// 32 BF16 with 256-row tiles (keeps the staging registers at 32 next to the
// 256 accumulators of a 128 x 128 wave tile).  Rows padded by 16 bytes.
template <class T, int BT>
struct Stage {
  static constexpr int BK = sizeof(T) == 4 ? 16 : (BT == 256 ? 32 : 64);
  static constexpr int ROW = BK + 16 / (int)sizeof(T);
};

// BT x BT tile per workgroup of four waves, each a (BT/2) x (BT/2) sub-tile.
// Pair-blocked epilogue: m = (p, c), n = (q, d) -> V2[(p*nq + q)][c][d] in the
// storage precision (FP32 -> BF16 by the hardware conversion, nearest even).
// FP32 16 x 16 accumulators: element r of a lane is D[4*(lane/16) + r][lane%16];
// mb and nbase are this lane's first row and column.  The byte offset splits
// into a row part (p*nq*kp + c*vu) and a column part (q*kp + d), both stepped
// without divisions in 32 bits (the host bounds the block below 4 GiB), so that
// every store is the uniform base plus one 32-bit offset.
template <class T, int TM, int TN>
__device__ inline void store_pairs(const LArgs& g, const f4 (&acc)[TM][TN], int64_t mb, int64_t nbase,
                                   bool interior = false) {
  constexpr uint32_t es = sizeof(T);
  const int vu = (int)g.vu;
  uint32_t coff[TN];
  bool cok[TN];
  {
    int q = (int)(nbase / vu), d = (int)(nbase % vu);
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      coff[j] = ((uint32_t)q * (uint32_t)g.kp + (uint32_t)d) * es;
      cok[j] = nbase + 16 * j < g.N;
      d += 16;
      while (d >= vu) {
        d -= vu;
        ++q;
      }
    }
  }
  const uint32_t pstep = (uint32_t)(g.nq * g.kp) * es, cstep = (uint32_t)vu * es;
  int p = (int)(mb / vu), c = (int)(mb % vu);
  char* V = (char*)g.C;
#pragma unroll
  for (int i = 0; i < TM; ++i) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      // row mb + 16 i + r: (p, c) advanced by one row from the previous r, by 13 across i
      const uint32_t ro = (uint32_t)p * pstep + (uint32_t)c * cstep;
      if (interior) {
#pragma unroll
        for (int j = 0; j < TN; ++j) *(T*)(V + (ro + coff[j])) = (T)acc[i][j][r];
      } else if (mb + 16 * i + r < g.M) {
#pragma unroll
        for (int j = 0; j < TN; ++j)
          if (cok[j]) *(T*)(V + (ro + coff[j])) = (T)acc[i][j][r];
      }
      c += r == 3 ? 13 : 1;
      while (c >= vu) {
        c -= vu;
        ++p;
      }
    }
  }
}

template <class T, int EPI, bool SPLIT, int BT = 128>
__global__ __launch_bounds__(NT) void gemm_lp_kernel(LArgs g) {
  constexpr int VL = Traits<T>::VL;
  constexpr int BK = Stage<T, BT>::BK;
  constexpr int KSTEP = Traits<T>::KSTEP;
  constexpr int ROW = Stage<T, BT>::ROW;
  constexpr int CPR = BK / VL;               // 16-byte chunks per row
  constexpr int CH = BT * CPR / NT;          // chunks per thread per operand
  constexpr int WM = BT / 2, WN = BT / 2;
  constexpr int TM = WM / 16, TN = WN / 16;
  __shared__ __attribute__((aligned(16))) T sA[2][BT * ROW];
  __shared__ __attribute__((aligned(16))) T sB[2][BT * ROW];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  int64_t tm, tn;
  if (EPI == EPI_PAIRS && g.skip_lower) {
    if (!diag_tile(blockIdx.x, (g.M + BT - 1) / BT, g.tiles_n, g.N, g.vu, BT, BT, tm, tn))
      return;  // whole workgroup, before any barrier
  } else {
    tile_of(blockIdx.x, (g.M + BT - 1) / BT, g.tiles_n, tm, tn);
  }
  const int64_t m0 = tm * BT, n0 = tn * BT;
  int64_t kbeg = 0, kend = g.K;
  if (SPLIT) {
    kbeg = (int64_t)blockIdx.z * g.kchunk;
    kend = kbeg + g.kchunk < g.K ? kbeg + g.kchunk : g.K;
  }
  const T* A = (const T*)g.A;
  const T* B = (const T*)g.B;

  // element offsets of this thread's 16-byte chunks, fixed over the K loop (-1: row
  // outside; the host guarantees M*lda and N*ldb below 2^31)
  int oa[CH], ob[CH];
#pragma unroll
  for (int c = 0; c < CH; ++c) {
    const int e = tid + c * NT;
    const int r = e / CPR, kc = (e % CPR) * VL;
    oa[c] = m0 + r < g.M ? (int)((m0 + r) * g.lda) + kc : -1;
    ob[c] = n0 + r < g.N ? (int)((n0 + r) * g.ldb) + kc : -1;
  }
  uint4 ra[CH], rb[CH];
  auto load = [&](int64_t k0) {
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int kc = ((tid + c * NT) % CPR) * VL;
      const int64_t kk = k0 + kc;
      ra[c] = (oa[c] >= 0 && kk < kend) ? load_chunk<T>(A + oa[c] + k0, kk, kend) : uint4{0u, 0u, 0u, 0u};
      rb[c] = (ob[c] >= 0 && kk < kend) ? load_chunk<T>(B + ob[c] + k0, kk, kend) : uint4{0u, 0u, 0u, 0u};
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int e = tid + c * NT;
      const int r = e / CPR, kc = (e % CPR) * VL;
      *reinterpret_cast<uint4*>(&sA[buf][r * ROW + kc]) = ra[c];
      *reinterpret_cast<uint4*>(&sB[buf][r * ROW + kc]) = rb[c];
    }
  };

  f4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};

  const int64_t nk = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
  if (nk > 0) {
    load(kbeg);
    store(0);
  }
  __syncthreads();
  const int lrow = lane >> 4, lcol = lane & 15;
  for (int64_t kt = 0; kt < nk; ++kt) {
    const int buf = (int)(kt & 1);
    if (kt + 1 < nk) load(kbeg + (kt + 1) * BK);
    const T* a_s = sA[buf];
    const T* b_s = sB[buf];
#pragma unroll
    for (int ks = 0; ks < BK / KSTEP; ++ks) {
      if constexpr (VL == 4) {
        // lane supplies A[m = lane%16][k = lane/16] and B[k = lane/16][n = lane%16]
        float af[TM], bf[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i) af[i] = a_s[(wm * WM + i * 16 + lcol) * ROW + ks * KSTEP + lrow];
#pragma unroll
        for (int j = 0; j < TN; ++j) bf[j] = b_s[(wn * WN + j * 16 + lcol) * ROW + ks * KSTEP + lrow];
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i], bf[j], acc[i][j], 0, 0, 0);
      } else {
        // lane supplies A[m = lane%16][k = 8*(lane/16) + e] and B[k = 8*(lane/16) + e][n = lane%16]
        bf8 af[TM], bf[TN];
#pragma unroll
        for (int i = 0; i < TM; ++i)
          af[i] = *reinterpret_cast<const bf8*>(&a_s[(wm * WM + i * 16 + lcol) * ROW + ks * KSTEP + lrow * 8]);
#pragma unroll
        for (int j = 0; j < TN; ++j)
          bf[j] = *reinterpret_cast<const bf8*>(&b_s[(wn * WN + j * 16 + lcol) * ROW + ks * KSTEP + lrow * 8]);
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bf[j], acc[i][j], 0, 0, 0);
      }
    }
    if (kt + 1 < nk) store(buf ^ 1);
    __syncthreads();
  }

  // FP32 16 x 16 accumulators: element r of a lane is D[4*(lane/16) + r][lane%16]
  const int64_t mb = m0 + wm * WM + 4 * lrow, nbase = n0 + wn * WN + lcol;
  if constexpr (EPI == EPI_PAIRS) {
    store_pairs<T, TM, TN>(g, acc, mb, nbase);
    return;
  }
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gm = mb + i * 16 + r;
        const int64_t gn = nbase + j * 16;
        if (gm >= g.M || gn >= g.N) continue;
        const float val = acc[i][j][r];
        if (EPI == EPI_SPLIT) {
          float* W = (float*)g.C + (SPLIT ? (int64_t)blockIdx.z * g.split_stride : 0);
          W[gm * g.N + gn] = val;
        } else {
          double* C = (double*)g.C;
          const int64_t off = g.c_nc ? gm * g.ldc + gn : gm + gn * g.ldc;
          double out = g.alpha * (double)val;
          if (g.beta != 0.0) out += g.beta * C[off];
          C[off] = out;
        }
      }
}

// ---------------------------------------------------------------------------
// Direct-to-LDS pair assembly (the ladder integral batches in FP32 or BF16).
// Both operands are K-contiguous rows; one LDS stage holds 128 bytes of K
// (32 FP32 or 64 BF16 elements) for the 128 rows of each operand tile, loaded
// straight from global memory (global_load_lds_dwordx4, 8 rows of 128 bytes
// per wave instruction).  Each lane fetches the 16-byte chunk that lands in
// its slot under slot = chunk ^ ((row >> 1) & 7), so that the 16 rows of a
// fragment read fall on distinct LDS banks.  A ring of S stages: a step waits
// for its own stage (S - 2 younger ones stay in flight), crosses a bare
// barrier, reads all its fragments with LDS reads that wait for their own
// results inside the asm block, issues the step S - 1 ahead, and runs its
// MFMAs.  Every fragment read brings 16 bytes of K per lane: BF16 feeds one
// 16x16x32 MFMA with it; FP32 feeds four 16x16x4 MFMAs, lane group g holding
// k = 16 b + 4 g + s in step s of block b (A and B use the same assignment).
// EPI_PAIRS writes the pair-blocked integrals; EPI_SPLIT writes FP32 partial
// products of the K chunk blockIdx.z (chunks a multiple of BK long) for a
// fixed-order reduction.  Requires 16-byte aligned operands and leading
// dimensions that are multiples of 8 elements.  A 16-byte chunk that starts
// below the end of its K range is loaded whole: K must be a multiple of the
// elements per 16 bytes, or each row must hold zeros up to that multiple.
typedef unsigned u4v __attribute__((ext_vector_type(4)));
// stages and 16-byte chunks per row and stage: BF16 two stages of 128-byte rows, FP32 three
// of 64-byte rows (measured at the 12864 x 12864 x 1200 ladder batches)
template <class T>
struct DlShape {
  static constexpr int S = sizeof(T) == 2 ? 2 : 3, CPR = sizeof(T) == 2 ? 8 : 4;
};

__device__ inline uint32_t lds_byte_address(const void* p) {
  return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void*)p;
}
constexpr int waitcnt_vm(int vm) { return (vm & 0xF) | ((vm >> 4) << 14) | (7 << 4) | (0xF << 8); }

// BT x BT output tile per workgroup: BT = 128 on four waves (2 x 2, 64 x 64 each) or
// BT = 256 on eight waves (2 x 4, 128 x 64 each), which halves the operand bytes per
// MFMA that the L2 has to supply.
template <int BT>
struct DlTile {
  static constexpr int NW = BT == 256 ? 8 : 4;   // waves
  static constexpr int WGN = NW / 2;             // waves along n
  static constexpr int WM = BT / 2, WN = BT / WGN;
  static constexpr int TM = WM / 16, TN = WN / 16;
};

template <class T, int S, int CPR, int EPI, int BT = 128>
__global__ __launch_bounds__(64 * DlTile<BT>::NW) void gemm_lp_dl_kernel(LArgs g) {
  constexpr int VL = Traits<T>::VL;          // elements per 16-byte chunk
  constexpr int RB = 16 * CPR;               // bytes of K per row and stage
  constexpr int BK = CPR * VL;               // elements of K per stage
  constexpr int H = CPR / 4;                 // fragment sub-steps per stage (4 chunks each)
  constexpr int RPI = 64 / CPR;              // rows per wave instruction
  constexpr int NW = DlTile<BT>::NW, WGN = DlTile<BT>::WGN;
  constexpr int IPW = BT / RPI / NW;         // instructions per operand per wave and stage
  constexpr int WM = DlTile<BT>::WM, WN = DlTile<BT>::WN, TM = DlTile<BT>::TM, TN = DlTile<BT>::TN;
  constexpr int STAGE = BT * RB;             // bytes per operand per stage
  static_assert(CPR == 4 || CPR == 8, "4 or 8 chunks per row");
  static_assert(TN == 4 && (TM == 4 || TM == 8), "wave tiles of 64 x 64 or 128 x 64");
  __shared__ __attribute__((aligned(16))) unsigned char sA[S][STAGE];
  __shared__ __attribute__((aligned(16))) unsigned char sB[S][STAGE];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave / WGN, wn = wave % WGN;
  int64_t tm, tn;
  int64_t zsplit = blockIdx.z;  // K chunk of a split product
  if (EPI == EPI_PAIRS && g.skip_lower) {
    if (!diag_tile(blockIdx.x, (g.M + BT - 1) / BT, g.tiles_n, g.N, g.vu, BT, BT, tm, tn))
      return;  // whole workgroup, before any barrier
  } else if (EPI == EPI_SPLIT && g.xcd_split) {
    // K chunks grouped per XCD: the tiles of one chunk share its operand rows in one L2
    zsplit = split_tile_of(blockIdx.x, (g.M + BT - 1) / BT, g.tiles_n, tm, tn);
  } else {
    tile_of(blockIdx.x, (g.M + BT - 1) / BT, g.tiles_n, tm, tn);
  }
  const int64_t m0 = tm * BT, n0 = tn * BT;
  int64_t kbeg = 0, kend = g.K;
  if (EPI == EPI_SPLIT) {
    kbeg = zsplit * g.kchunk;
    kend = kbeg + g.kchunk < g.K ? kbeg + g.kchunk : g.K;
  }
  const T* A = (const T*)g.A;
  const T* B = (const T*)g.B;
  const T* zrow = (const T*)lp_zero_row;
  // swizzle of a row: 8 chunks use (row >> 1) & 7, 4 chunks (row >> 2) & 3
  auto swz = [](int r) { return CPR == 8 ? (r >> 1) & 7 : (r >> 2) & 3; };
  // wave instruction q covers rows RPI*q .. RPI*q + RPI-1; lane l takes row RPI*q + l/CPR
  // and the chunk that lands in slot l % CPR
  auto issue = [&](int slot, int64_t k0) {
#pragma unroll
    for (int qi = 0; qi < IPW; ++qi) {
      const int q = wave * IPW + qi;
      const int r = q * RPI + lane / CPR;
      const int chunk = (lane % CPR) ^ swz(r);
      const int64_t k = k0 + chunk * VL;
      const T* sa = (m0 + r < g.M && k < kend) ? A + (m0 + r) * g.lda + k : zrow;
      const T* sb = (n0 + r < g.N && k < kend) ? B + (n0 + r) * g.ldb + k : zrow;
      const int dst = q * RPI * RB;
      __builtin_amdgcn_global_load_lds((const void*)sa, (void __attribute__((address_space(3)))*)&sA[slot][dst], 16, 0,
                                       0);
      __builtin_amdgcn_global_load_lds((const void*)sb, (void __attribute__((address_space(3)))*)&sB[slot][dst], 16, 0,
                                       0);
    }
  };
  f4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  const int lrow = lane >> 4, lcol = lane & 15;
  // byte offset of this lane's fragment for sub-step h (chunk 4h + lane/16) of row block 0;
  // the swizzle of rows base + lcol depends on lcol only (the bases are multiples of 16), and
  // the next 16 rows lie 16 * RB bytes on
  uint32_t ao[H], bo[H];
#pragma unroll
  for (int h = 0; h < H; ++h) {
    ao[h] = (uint32_t)((wm * WM + lcol) * RB + (((4 * h + lrow) ^ swz(lcol)) * 16));
    bo[h] = (uint32_t)((wn * WN + lcol) * RB + (((4 * h + lrow) ^ swz(lcol)) * 16));
  }
  const int64_t nk = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
#pragma unroll
  for (int t = 0; t < S - 1; ++t) issue(t, kbeg + (int64_t)t * BK);
  int slot = 0, fill = S - 1;  // stage read this step, stage refilled this step
  for (int64_t kt = 0; kt < nk; ++kt) {
    __builtin_amdgcn_s_waitcnt(waitcnt_vm(2 * IPW * (S - 2)));
    __builtin_amdgcn_s_barrier();
    const uint32_t sa = lds_byte_address(sA[slot]), sb = lds_byte_address(sB[slot]);
    if constexpr (TM == 4) {
      u4v af[H][TM], bf[H][TN];
#pragma unroll
      for (int h = 0; h < H; ++h) {
        const uint32_t pa = sa + ao[h], pb = sb + bo[h];
        asm volatile(
            "ds_read_b128 %0, %8\n"
            "ds_read_b128 %1, %8 offset:%10\n"
            "ds_read_b128 %2, %8 offset:%11\n"
            "ds_read_b128 %3, %8 offset:%12\n"
            "ds_read_b128 %4, %9\n"
            "ds_read_b128 %5, %9 offset:%10\n"
            "ds_read_b128 %6, %9 offset:%11\n"
            "ds_read_b128 %7, %9 offset:%12\n"
            "s_waitcnt lgkmcnt(0)"
            : "=&v"(af[h][0]), "=&v"(af[h][1]), "=&v"(af[h][2]), "=&v"(af[h][3]), "=&v"(bf[h][0]), "=&v"(bf[h][1]),
              "=&v"(bf[h][2]), "=&v"(bf[h][3])
            : "v"(pa), "v"(pb), "n"(16 * RB), "n"(32 * RB), "n"(48 * RB)
            : "memory");
      }
      issue(fill, kbeg + (kt + S - 1) * BK);  // past the K range: zero rows
      slot = slot + 1 == S ? 0 : slot + 1;
      fill = fill + 1 == S ? 0 : fill + 1;
#pragma unroll
      for (int h = 0; h < H; ++h)
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) {
            if constexpr (VL == 8) {
              acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                  __builtin_bit_cast(bf8, af[h][i]), __builtin_bit_cast(bf8, bf[h][j]), acc[i][j], 0, 0, 0);
            } else {
              const f4 a = __builtin_bit_cast(f4, af[h][i]), b = __builtin_bit_cast(f4, bf[h][j]);
#pragma unroll
              for (int e = 0; e < 4; ++e)
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[e], b[e], acc[i][j], 0, 0, 0);
            }
          }
    } else {
      // 128 x 64 wave tiles: each sub-step's fragments are read just before its MFMAs, in two
      // groups: the four B fragments with the first four A fragments, whose 16 MFMAs then run
      // while the other four A fragments are read (48 fragment registers; each accumulator
      // takes the same MFMAs in the same order as with one group of 12 reads)
#pragma unroll
      for (int h = 0; h < H; ++h) {
        u4v af[TM], bf[TN];
        const uint32_t pa = sa + ao[h], pb = sb + bo[h];
        asm volatile(
            "ds_read_b128 %0, %8\n"
            "ds_read_b128 %1, %8 offset:%10\n"
            "ds_read_b128 %2, %8 offset:%11\n"
            "ds_read_b128 %3, %8 offset:%12\n"
            "ds_read_b128 %4, %9\n"
            "ds_read_b128 %5, %9 offset:%10\n"
            "ds_read_b128 %6, %9 offset:%11\n"
            "ds_read_b128 %7, %9 offset:%12\n"
            "s_waitcnt lgkmcnt(0)"
            : "=&v"(af[0]), "=&v"(af[1]), "=&v"(af[2]), "=&v"(af[3]), "=&v"(bf[0]), "=&v"(bf[1]), "=&v"(bf[2]),
              "=&v"(bf[3])
            : "v"(pa), "v"(pb), "n"(16 * RB), "n"(32 * RB), "n"(48 * RB)
            : "memory");
        if (h == 0) {  // every wave has read the stage's first fragments: refill the oldest stage
          issue(fill, kbeg + (kt + S - 1) * BK);  // past the K range: zero rows
          slot = slot + 1 == S ? 0 : slot + 1;
          fill = fill + 1 == S ? 0 : fill + 1;
        }
        auto mma = [&](int i0) {
#pragma unroll
          for (int i = i0; i < i0 + 4; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
              if constexpr (VL == 8) {
                acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, af[i]),
                                                                    __builtin_bit_cast(bf8, bf[j]), acc[i][j], 0, 0, 0);
              } else {
                const f4 a = __builtin_bit_cast(f4, af[i]), b = __builtin_bit_cast(f4, bf[j]);
#pragma unroll
                for (int e = 0; e < 4; ++e)
                  acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[e], b[e], acc[i][j], 0, 0, 0);
              }
            }
        };
        mma(0);
        asm volatile(
            "ds_read_b128 %0, %4 offset:%5\n"
            "ds_read_b128 %1, %4 offset:%6\n"
            "ds_read_b128 %2, %4 offset:%7\n"
            "ds_read_b128 %3, %4 offset:%8\n"
            "s_waitcnt lgkmcnt(0)"
            : "=&v"(af[4]), "=&v"(af[5]), "=&v"(af[6]), "=&v"(af[7])
            : "v"(pa), "n"(64 * RB), "n"(80 * RB), "n"(96 * RB), "n"(112 * RB)
            : "memory");
        mma(4);
      }
    }
  }
  __builtin_amdgcn_s_waitcnt(0);  // the last (zero) stages have landed before the wave retires
  const int64_t mb = m0 + wm * WM + 4 * lrow, nbase = n0 + wn * WN + lcol;
  if constexpr (EPI == EPI_PAIRS) {
    // interior wave tiles (every row and column in range) store without checks
    const bool interior = m0 + wm * WM + WM <= g.M && n0 + wn * WN + WN <= g.N;
    store_pairs<T, TM, TN>(g, acc, mb, nbase, interior);
  } else if constexpr (EPI == EPI_F64) {
    double* C = (double*)g.C;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gm = mb + i * 16 + r;
        if (gm >= g.M) continue;
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          const int64_t gn = nbase + j * 16;
          if (gn >= g.N) continue;
          const int64_t off = g.c_nc ? gm * g.ldc + gn : gm + gn * g.ldc;
          double out = g.alpha * (double)acc[i][j][r];
          if (g.beta != 0.0) out += g.beta * C[off];
          C[off] = out;
        }
      }
  } else {
    float* W = (float*)g.C + zsplit * g.split_stride;
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gm = mb + i * 16 + r;
        if (gm >= g.M) continue;
#pragma unroll
        for (int j = 0; j < TN; ++j)
          if (nbase + j * 16 < g.N) W[gm * g.N + nbase + j * 16] = acc[i][j][r];
      }
  }
}

// C(m,n) = alpha * sum_z W[z][m*N + n] + beta * C(m,n), summed in FP64 in z order.
__global__ void lp_split_reduce(const float* W, double* C, int64_t M, int64_t N, int nsplit, int64_t ldc, int c_nc,
                                double alpha, double beta) {
  const int64_t MN = M * N;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < MN;
       idx += (int64_t)gridDim.x * blockDim.x) {
    double sum = 0.0;
    for (int z = 0; z < nsplit; ++z) sum += (double)W[z * MN + idx];
    const int64_t m = idx / N, nn = idx % N;
    const int64_t off = c_nc ? m * ldc + nn : m + nn * ldc;
    double out = alpha * sum;
    if (beta != 0.0) out += beta * C[off];
    C[off] = out;
  }
}

// dst[r*ldd + c] = round(src[i] - sub[i]), i = r*sr + c*sc (sub may be NULL),
// through a 64 x 64 LDS tile; the source is read along whichever of its axes
// is contiguous.
template <class T>
__global__ __launch_bounds__(256) void lp_convert_kernel(T* dst, int64_t ldd, const double* src, const double* sub,
                                                         int64_t rows, int64_t cols, int64_t sr, int64_t sc,
                                                         int64_t tiles_c) {
  __shared__ double tile[64][65];
  const int64_t r0 = ((int64_t)blockIdx.x / tiles_c) * 64, c0 = ((int64_t)blockIdx.x % tiles_c) * 64;
  const int tid = threadIdx.x;
  const bool row_major_src = sc == 1;
  for (int e = tid; e < 64 * 64; e += 256) {
    const int a = e / 64, b = e % 64;  // consecutive threads vary b
    const int rr = row_major_src ? a : b, cc = row_major_src ? b : a;
    const int64_t r = r0 + rr, c = c0 + cc;
    double x = 0.0;
    if (r < rows && c < cols) {
      const int64_t i = r * sr + c * sc;
      x = sub ? src[i] - sub[i] : src[i];
    }
    tile[rr][cc] = x;
  }
  __syncthreads();
  // the row padding up to the next multiple of 64 columns (within ldd) is written as zeros, so
  // that GEMMs may load whole 16-byte chunks past the end of K
  for (int e = tid; e < 64 * 64; e += 256) {
    const int rr = e / 64, cc = e % 64;
    const int64_t r = r0 + rr, c = c0 + cc;
    if (r < rows && c < ldd) dst[r * ldd + c] = c < cols ? lp_round<T>((float)tile[rr][cc]) : (T)0.0f;
  }
}

unsigned nb(int64_t total) {
  int64_t b = (total + 255) / 256;
  if (b > (1 << 20)) b = 1 << 20;
  return (unsigned)(b < 1 ? 1 : b);
}

template <class T>
void launch_convert(void* dst, int64_t ldd, const double* src, const double* sub, int64_t rows, int64_t cols,
                    int64_t sr, int64_t sc, hipStream_t s) {
  const int64_t tr = (rows + 63) / 64, tc = (cols + 63) / 64;
  if (tr * tc <= 0) return;
  if (tr * tc >= ((int64_t)1 << 31)) throw ArgError("conversion too large");
  hipLaunchKernelGGL(lp_convert_kernel<T>, dim3((unsigned)(tr * tc)), dim3(256), 0, s, (T*)dst, ldd, src, sub, rows,
                     cols, sr, sc, tc);
  DCSD_CHECK_LAUNCH();
}

template <class T>
void launch_gemm(const LpGemm& q, hipStream_t s) {
  LArgs a{};
  a.M = q.M; a.N = q.N; a.K = q.K;
  a.A = q.A; a.lda = q.lda; a.B = q.B; a.ldb = q.ldb;
  a.alpha = q.alpha; a.beta = q.beta;
  a.tiles_n = (q.N + TILE - 1) / TILE;
  const int64_t tiles = ((q.M + TILE - 1) / TILE) * a.tiles_n;
  // direct-to-LDS when whole 16-byte chunks may be loaded up to the end of K
  constexpr int DBK = DlShape<T>::CPR * Traits<T>::VL;
  const bool dl = q.k_padded || q.K % Traits<T>::VL == 0;
  if (q.ks <= 1) {
    a.C = q.C; a.ldc = q.ldc; a.c_nc = q.c_nc ? 1 : 0;
    a.kchunk = q.K;
    // BF16 products with at least one 256 x 256 tile per compute unit (the ring and delta
    // products of the residual): 256 x 256 tiles on eight waves
    const int64_t t256 = ((q.M + 255) / 256) * ((q.N + 255) / 256);
    if (dl && sizeof(T) == 2 && t256 >= 256 && q.K >= 1024) {
      a.tiles_n = (q.N + 255) / 256;
      hipLaunchKernelGGL((gemm_lp_dl_kernel<T, DlShape<T>::S, DlShape<T>::CPR, EPI_F64, 256>), dim3((unsigned)t256),
                         dim3(64 * DlTile<256>::NW), 0, s, a);
      DCSD_CHECK_LAUNCH();
      return;
    }
    if (dl)
      hipLaunchKernelGGL((gemm_lp_dl_kernel<T, DlShape<T>::S, DlShape<T>::CPR, EPI_F64>), dim3((unsigned)tiles), dim3(NT),
                         0, s, a);
    else
      hipLaunchKernelGGL((gemm_lp_kernel<T, EPI_F64, false>), dim3((unsigned)tiles), dim3(NT), 0, s, a);
    DCSD_CHECK_LAUNCH();
    return;
  }
  const int64_t step = dl ? std::max<int64_t>(DBK, Stage<T, TILE>::BK) : Stage<T, TILE>::BK;
  int64_t chunk = (q.K + q.ks - 1) / q.ks;
  chunk = (chunk + step - 1) / step * step;
  const int ks = (int)((q.K + chunk - 1) / chunk);
  a.C = q.work;
  a.kchunk = chunk;
  a.split_stride = q.M * q.N;
  if (dl && q.big_tiles && sizeof(T) == 2) {
    a.tiles_n = (q.N + 255) / 256;
    const int64_t t256 = ((q.M + 255) / 256) * a.tiles_n;
    a.xcd_split = ks % 8 == 0 ? 1 : 0;
    if (a.xcd_split)
      hipLaunchKernelGGL((gemm_lp_dl_kernel<T, DlShape<T>::S, DlShape<T>::CPR, EPI_SPLIT, 256>),
                         dim3((unsigned)(t256 * ks)), dim3(64 * DlTile<256>::NW), 0, s, a);
    else
      hipLaunchKernelGGL((gemm_lp_dl_kernel<T, DlShape<T>::S, DlShape<T>::CPR, EPI_SPLIT, 256>),
                         dim3((unsigned)t256, 1, (unsigned)ks), dim3(64 * DlTile<256>::NW), 0, s, a);
  } else if (dl) {
    a.xcd_split = ks % 8 == 0 ? 1 : 0;
    const dim3 grid = a.xcd_split ? dim3((unsigned)(tiles * ks)) : dim3((unsigned)tiles, 1, (unsigned)ks);
    hipLaunchKernelGGL((gemm_lp_dl_kernel<T, DlShape<T>::S, DlShape<T>::CPR, EPI_SPLIT>), grid, dim3(NT), 0, s, a);
  } else
    hipLaunchKernelGGL((gemm_lp_kernel<T, EPI_SPLIT, true>), dim3((unsigned)tiles, 1, (unsigned)ks), dim3(NT), 0, s, a);
  DCSD_CHECK_LAUNCH();
  hipLaunchKernelGGL(lp_split_reduce, dim3(nb(q.M * q.N)), dim3(256), 0, s, (const float*)q.work, q.C, q.M, q.N, ks,
                     q.ldc, q.c_nc ? 1 : 0, q.alpha, q.beta);
  DCSD_CHECK_LAUNCH();
}

template <class T, int BT>
void launch_pairs(const void* BlT, int64_t ldk, int64_t naux, int64_t vu, int64_t p0, int64_t np, int64_t q0,
                  int64_t nq, int64_t kp, void* V2, hipStream_t s) {
  LArgs a{};
  a.M = np * vu; a.N = nq * vu; a.K = naux;
  a.A = (const T*)BlT + p0 * vu * ldk; a.lda = ldk;
  a.B = (const T*)BlT + q0 * vu * ldk; a.ldb = ldk;
  a.C = V2; a.vu = vu; a.nq = nq; a.kp = kp;
  a.kchunk = naux;
  a.tiles_n = (a.N + BT - 1) / BT;
  const int64_t tiles_m = (a.M + BT - 1) / BT;
  // a diagonal batch is symmetric under (p, c) <-> (q, d): the tiles entirely in p > q are
  // skipped and those pairs copied from their mirrors below
  a.skip_lower = p0 == q0 && np == nq && np * (np - 1) / 2 <= 65535 && diag_skips(np, vu, BT, BT);
  const int64_t tiles = a.skip_lower ? diag_grid(tiles_m, a.tiles_n) : tiles_m * a.tiles_n;
  if (naux % Traits<T>::VL == 0)
    hipLaunchKernelGGL((gemm_lp_dl_kernel<T, DlShape<T>::S, DlShape<T>::CPR, EPI_PAIRS, BT>), dim3((unsigned)tiles),
                       dim3(64 * DlTile<BT>::NW), 0, s, a);
  else
    hipLaunchKernelGGL((gemm_lp_kernel<T, EPI_PAIRS, false, BT>), dim3((unsigned)tiles), dim3(NT), 0, s, a);
  DCSD_CHECK_LAUNCH();
  if (a.skip_lower) {
    const int t = (int)((vu + 31) / 32);
    hipLaunchKernelGGL(pair_mirror_kernel<T>, dim3((unsigned)(t * t), (unsigned)(np * (np - 1) / 2)), dim3(256), 0, s,
                       (T*)V2, vu, kp, np, t);
    DCSD_CHECK_LAUNCH();
  }
}

void check_lp(const LpGemm& q) {
  if (q.M <= 0 || q.N <= 0 || q.K <= 0) throw ArgError("low-precision GEMM: empty shape");
  if (q.M * q.lda >= ((int64_t)1 << 31) || q.N * q.ldb >= ((int64_t)1 << 31))
    throw ArgError("low-precision GEMM: operand too large for 32-bit offsets");
  if (q.lda % 8 || q.ldb % 8 || q.lda < q.K || q.ldb < q.K) throw ArgError("low-precision GEMM: bad leading dimension");
  if (((uintptr_t)q.A | (uintptr_t)q.B) & 15) throw ArgError("low-precision GEMM: operands not 16-byte aligned");
  if (q.ks > 1 && !q.work) throw ArgError("low-precision GEMM: split-K needs a workspace");
}

}  // namespace

size_t lp_size(int precision) { return precision == DCSD_PREC_BF16 ? 2 : 4; }

void lp_convert(int precision, void* dst, int64_t ldd, const double* src, const double* sub, int64_t rows,
                int64_t cols, int64_t sr, int64_t sc, hipStream_t s) {
  if (precision == DCSD_PREC_BF16)
    launch_convert<__bf16>(dst, ldd, src, sub, rows, cols, sr, sc, s);
  else
    launch_convert<float>(dst, ldd, src, sub, rows, cols, sr, sc, s);
}

void lp_gemm(const LpGemm& q, hipStream_t s) {
  check_lp(q);
  if (q.precision == DCSD_PREC_BF16)
    launch_gemm<__bf16>(q, s);
  else
    launch_gemm<float>(q, s);
}

void lp_pairs(int precision, const void* BlT, int64_t ldk, int64_t naux, int64_t vu, int64_t p0, int64_t np,
              int64_t q0, int64_t nq, int64_t kp, void* V2, hipStream_t s) {
  if (ldk % 8 || kp % 8) throw ArgError("low-precision ladder: bad leading dimension");
  if ((p0 + np) * vu * ldk >= ((int64_t)1 << 31) || (q0 + nq) * vu * ldk >= ((int64_t)1 << 31))
    throw ArgError("low-precision ladder: factor too large for 32-bit offsets");
  if (np * nq * kp * (int64_t)lp_size(precision) >= ((int64_t)1 << 32))
    throw ArgError("low-precision ladder: integral block too large for 32-bit offsets");
  // BF16 batches of at least 512 rows take 256 x 256 tiles (eight waves): at BF16 rates the
  // 128 x 128 tiles asked more operand bytes of the L2 per MFMA than it delivered
  if (precision == DCSD_PREC_BF16 && np * vu >= 512 && nq * vu >= 512)
    launch_pairs<__bf16, 256>(BlT, ldk, naux, vu, p0, np, q0, nq, kp, V2, s);
  else if (precision == DCSD_PREC_BF16)
    launch_pairs<__bf16, 128>(BlT, ldk, naux, vu, p0, np, q0, nq, kp, V2, s);
  else
    launch_pairs<float, 128>(BlT, ldk, naux, vu, p0, np, q0, nq, kp, V2, s);
}

}  // namespace dcsd
