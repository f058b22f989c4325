// Operation tape for the reverse-mode (adjoint) sweep of the residual and of
// the constants built from (B, F) (internal).
//
// While a tape is active, every device operation of the forward code goes
// through a recording wrapper that stores the operation with its original
// pointers and executes it.  Operands whose values the adjoint needs (GEMM
// operands, the inputs of the bilinear ladder back-transformation, the
// coupling and the energy) are snapshotted when their buffer may still be
// overwritten; buffers flagged constant for the tape are referenced in place.
// The backward sweep walks the tape in reverse and applies the hand-written
// adjoint of each operation to shadow ("bar") buffers of the same layout.
#pragma once

#include <cstdint>
#include <vector>

#include "common.h"

namespace dcsd {

struct Ctx;

enum OpKind : int {
  OP_GEMM = 0,   // C = alpha op(A) op(B) + beta C (GemmArgs)
  OP_COPY,       // strided dst = alpha src + beta dst
  OP_FILL,       // p[0..n) = value
  OP_AXPBY,      // y = a x + b y
  OP_MEMCPY,     // dst = src (device to device)
  OP_UPLOAD,     // dst = host constant (no derivative)
  OP_SWAPTU,     // dst = swap_tu(src)
  OP_JVEC,       // J[P] = sum_{k<o} Ba[P,k,k] + Bb[P,k,k]
  OP_BREDUCE,    // dst += alpha sum_b src[b]
  OP_STACK,      // ladder amplitude stack from t2
  OP_LADDER,     // spatial ladder result Rp from the stack (blocks recomputed in the sweep)
  OP_MTRANS,     // R2 += T1 back-transformation of Rp
  OP_COUPLING,   // R -= K(T) W
  OP_ENERGY      // E_A(T) into a scalar
};

struct TapeOp {
  int kind = 0;
  GemmArgs g;                       // OP_GEMM (original pointers)
  const double* Aval = nullptr;     // values of A / B at the time of the operation
  const double* Bval = nullptr;
  Strided st{};                     // OP_COPY
  double alpha = 0.0, beta = 0.0;
  double* dst = nullptr;
  const double* src = nullptr;
  const double* src2 = nullptr;
  const double* val[4] = {nullptr, nullptr, nullptr, nullptr};  // value snapshots of special operations
  int64_t n = 0;
  int64_t i64[6] = {0, 0, 0, 0, 0, 0};
  int ints[6] = {0, 0, 0, 0, 0, 0};
};

struct Snapshot {
  int buf;
  int version;
  const double* lo;
  const double* hi;
  double* copy;
};

struct Tape {
  std::vector<TapeOp> ops;
  std::vector<Snapshot> snaps;
  std::vector<double*> scratch;  // device memory owned by the tape (snapshots taken while sizing)
  int64_t temp_need = 0;         // largest temporary (doubles) the sweep needs
  // Snapshot memory reserved by the context: once `arena` is set, snapshots are
  // carved from it (256-byte aligned) and nothing is allocated; `need` is the
  // arena size the last recording required.
  double* arena = nullptr;
  int64_t arena_cap = 0, arena_used = 0, need = 0;
  void clear();
};

// The tape being recorded on this thread (null when not recording).
inline thread_local Tape* t_tape = nullptr;
inline thread_local Ctx* t_ctx = nullptr;

// Recording hooks (defined in adjoint.cpp); each returns after recording, the
// caller executes the operation.
void tape_gemm(const GemmArgs& g);
void tape_copy(double* dst, const double* src, const Strided& st, double alpha, double beta);
void tape_simple(int kind, double* dst, const double* src, int64_t n, double a, double b);
void tape_op(const TapeOp& op);
// Value of a device range needed by an adjoint: the pointer itself if its
// buffer cannot change before the sweep, otherwise a snapshot copy.
const double* tape_value(const double* p, int64_t count);

}  // namespace dcsd
