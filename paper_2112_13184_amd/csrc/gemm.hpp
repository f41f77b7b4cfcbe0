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
// out[0 .. n) = 0 (n <= 64) by a kernel (no memset node in captured graphs).
void clear_words(hipStream_t st, unsigned* out, int n);

// ---------------------------------------------------------------------------
// Operands stored once in the reduced type (BF16, or split FP16 as a hi and a
// lo plane), for products that read the same large operand many times (the
// corners of the randomized SVD).  A pre-converted operand is `rows` rows of
// ld values with k contiguous; ld is a multiple of 32 and the values past the
// logical K are zero, so that every 32-wide k-tile is whole.
//   BF16:  x -> bf16(float(x)).
//   F16:   x * sc = hi + 2^-11 lo (hi, lo FP16), sc a power of two: one per
//          operand (from `amax`, FP32 bits of its largest |entry|) or one per
//          row (`rowscale`, FP32 powers of two), undone in the product.
// ---------------------------------------------------------------------------
struct PreOperand {
  const void* p = nullptr;     // hi plane of problem 0 (2-byte values)
  long ld = 0;                 // row pitch (multiple of 32)
  long bs = 0;                 // batch stride (elements)
  long lo = 0;                 // F16: lo plane at p + lo (elements)
  const unsigned* amax = nullptr;   // F16: per-operand scale source
  const float* rowscale = nullptr;  // F16: per-row scales [batch][rows] (overrides amax)
  long rs_bs = 0;
};

// Padded row pitch of a pre-converted operand of logical width K.
inline long pre_ld(long K) { return ((K + 31) / 32) * 32; }

// out <- G_b (row-major n x n, batch stride gbs) and G_b^T, pre-converted:
// problem b holds [G rows (n x ld)][G^T rows (n x ld)] at out + b * obs (hi
// planes; F16 lo planes at + lo).  F16 scales by the power of two of *amax.
void convert_square_pre(hipStream_t st, GemmType type, const double* G, long gbs, int n, int batch, void* out,
                        long obs, long lo, const unsigned* amax);
// out <- the k columns of the column-major n x k panels X_b (ld n, batch
// stride xbs) as k pre-converted rows of pre_ld(n) values at out + b * obs.
// F16: one power-of-two scale per column -> rowscale[b * rs_bs + j].
void convert_panel_pre(hipStream_t st, GemmType type, const double* X, long xbs, int n, int k, int batch, void* out,
                       long obs, long lo, float* rowscale, long rs_bs);

// out <- the C columns of the row-major R x C matrices src_b (leading
// dimension lds, batch stride sbs) as C pre-converted rows of pre_ld(R)
// values at out + b * obs (R <= 320).  F16: one power-of-two scale per
// output row -> rowscale[b * rs_bs + c].
void convert_cols_pre(hipStream_t st, GemmType type, const double* src, long lds, long sbs, int R, int C, int batch,
                      void* out, long obs, long lo, float* rowscale, long rs_bs);

// C = alpha * A B^T: A (M x Kp) and B (N x Kp) pre-converted (type BF16 or
// F16), FP32 accumulation, C FP64 (any strides); Kp = the common row pitch's
// logical width rounded to 32.
void gemm_pre(hipStream_t st, GemmType type, int M, int N, int Kp, double alpha, const PreOperand& A,
              const PreOperand& B, const OutOperand& C, int batch, const GemmWorkspace& ws);


}  // namespace ctm
