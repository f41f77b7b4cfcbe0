// Generic MFMA GEMM with strided or table-addressed operands.
//
// Every contraction of the CTMRG sweep is written as C = alpha * A * B + beta * C
// where each operand element (i, j) lives at
//     base + batch * bs + (t0 ? t0[i] : i * s0) + (t1 ? t1[j] : j * s1).
// Plain, transposed and batched GEMMs use strides; the single-layer ket / bra
// absorption, whose row and column indices are products of a chi index and
// bond indices, uses separable offset tables so that the index permutation
// happens in the loads and stores instead of in separate transpose passes.
#pragma once

#include "common.hpp"

namespace ctm {

struct Operand {
  const void* p = nullptr;
  long s0 = 0, s1 = 0;       // strides of the row / column index
  const int* t0 = nullptr;   // row offset table (overrides s0)
  const int* t1 = nullptr;   // column offset table (overrides s1)
  long bs = 0;               // batch stride
};

struct OutOperand {
  void* p = nullptr;
  long s0 = 0, s1 = 0;
  const int* t0 = nullptr;
  const int* t1 = nullptr;
  long bs = 0;
};

inline Operand rowmajor(const void* p, long ld, long bs = 0) { Operand o; o.p = p; o.s0 = ld; o.s1 = 1; o.bs = bs; return o; }
inline Operand colmajor(const void* p, long ld, long bs = 0) { Operand o; o.p = p; o.s0 = 1; o.s1 = ld; o.bs = bs; return o; }
inline OutOperand out_rowmajor(void* p, long ld, long bs = 0) { OutOperand o; o.p = p; o.s0 = ld; o.s1 = 1; o.bs = bs; return o; }
inline OutOperand out_colmajor(void* p, long ld, long bs = 0) { OutOperand o; o.p = p; o.s0 = 1; o.s1 = ld; o.bs = bs; return o; }

// Element type of A and B.  Accumulation is FP64 for F64 and FP32 otherwise;
// C is always FP64.  For the reduced types the operands are converted (round
// to nearest even) while being staged into LDS.
enum class GemmType { F64 = 0, F32 = 1, BF16 = 2, F16 = 3 };

struct GemmWorkspace {
  double* p = nullptr;   // split-K partial sums
  size_t elems = 0;
};

// C = alpha * A(MxK) * B(KxN) + beta * C for `batch` independent problems.
// A and B are FP64 in memory.  `type` selects the arithmetic of the
// multiply: F64 (MFMA f64), F32 / BF16 (one MFMA pass), F16 (FP16 split into
// hi + lo parts, three MFMA passes).
void gemm(hipStream_t st, GemmType type, int M, int N, int K, double alpha, const Operand& A,
          const Operand& B, double beta, const OutOperand& C, int batch, const GemmWorkspace& ws);

// Workspace elements gemm() may need for this shape (0 if no split-K).
size_t gemm_workspace_elems(int M, int N, int K, int batch);

}  // namespace ctm
