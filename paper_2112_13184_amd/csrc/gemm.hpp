// Generic MFMA GEMM with strided or table-addressed operands.
//
// Every contraction of the CTMRG sweep is written as C = alpha * A * B + beta * C
// where each operand element (i, j) lives at
//     base + batch * bs + (t0 ? t0[i] : i * s0) + (t1 ? t1[j] : j * s1),
// or, for batches whose problems are not evenly spaced (the corners and
// tensors of different sites), base + bo[batch] + (row and column offsets)
// with bo a device array of one element offset per problem.
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
  const long* bo = nullptr;  // per-problem element offsets from p (device; override bs)
  const unsigned* amax = nullptr;   // split FP16: largest |entry| over the batch
                                    // (FP32 bits, device), else scanned per call
};

struct OutOperand {
  void* p = nullptr;
  long s0 = 0, s1 = 0;
  const int* t0 = nullptr;
  const int* t1 = nullptr;
  long bs = 0;
  const long* bo = nullptr;  // per-problem element offsets from p (device; override bs)
};

inline Operand rowmajor(const void* p, long ld, long bs = 0) { Operand o; o.p = p; o.s0 = ld; o.s1 = 1; o.bs = bs; return o; }
inline Operand colmajor(const void* p, long ld, long bs = 0) { Operand o; o.p = p; o.s0 = 1; o.s1 = ld; o.bs = bs; return o; }
inline OutOperand out_rowmajor(void* p, long ld, long bs = 0) { OutOperand o; o.p = p; o.s0 = ld; o.s1 = 1; o.bs = bs; return o; }
inline OutOperand out_colmajor(void* p, long ld, long bs = 0) { OutOperand o; o.p = p; o.s0 = 1; o.s1 = ld; o.bs = bs; return o; }

// Arithmetic of the multiply.  Accumulation is FP64 for F64 and FP32
// otherwise; A, B and C are FP64 in memory.  For the reduced types the
// operands are rounded (to nearest even) while being staged into LDS:
//   F32  one v_mfma_f32_16x16x4f32 pass;
//   BF16 one v_mfma_f32_16x16x32_bf16 pass;
//   F16  split FP16: x * 2^s = hi + 2^-11 lo with hi, lo FP16 and one power
//        of two s per operand (from its largest entry, so that it fits FP16's
//        range), three v_mfma_f32_16x16x32_f16 passes (hi hi, hi lo, lo hi)
//        with the correction accumulated apart (Markidis et al. 2018, Ootomo
//        and Yokota 2022).
enum class GemmType { F64 = 0, F32 = 1, BF16 = 2, F16 = 3 };

struct GemmWorkspace {
  double* p = nullptr;       // split-K partial sums
  size_t elems = 0;
  unsigned* amax = nullptr;  // 2 words: largest |A| and |B| (F16 scaling)
};

// C = alpha * A(MxK) * B(KxN) + beta * C for `batch` independent problems,
// in the arithmetic `type` selects (F16 needs ws.amax).
void gemm(hipStream_t st, GemmType type, int M, int N, int K, double alpha, const Operand& A,
          const Operand& B, double beta, const OutOperand& C, int batch, const GemmWorkspace& ws);

// *out = largest |entry| (FP32 bits) of an R x C operand over `batch` problems.
void operand_amax(hipStream_t st, const Operand& P, int R, int C, int batch, unsigned* out);


}  // namespace ctm
