// MFMA GEMM for gfx950 with strided / table-addressed operands (see gemm.hpp).
//
// Tiling: 256 threads = 4 wave64s per workgroup, output tile BM x BN, K step
// BK = 16 (FP64).  A and B tiles are staged through LDS as As[m][k] and
// Bs[n][k] (k contiguous, one padding element per row so that both the
// transposing stores and the MFMA fragment reads are free of bank conflicts),
// double buffered: while the MFMAs of k-tile t run on one buffer, tile t + 1
// is stored from registers into the other and, in the FP64 and FP32 kernels,
// the loads of tile t + 2 are in flight into a second register set (the two
// sets alternate; the main loop is unrolled by two).  Each wave owns a
// WM x WN sub-tile of 16x16 MFMA blocks.
//
// FP64 uses v_mfma_f64_16x16x4f64: lane l supplies A[l%16][k] and B[k][l%16]
// for k-slot l/16, and holds D[(l/16) + 4r][l%16] in register r.  Within a K
// step of 16 the four MFMAs take k = 4*(l/16) + s (s = 0..3), so each lane
// reads its four A (B) values as one contiguous 32-byte LDS run.
#include "gemm.hpp"

#include <algorithm>
#include <type_traits>

namespace ctm {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

struct KArgs {
  const double* A;
  const double* B;
  double* C;
  long sa0, sa1, sb0, sb1, sc0, sc1;
  const int *ta0, *ta1, *tb0, *tb1, *tc0, *tc1;
  long bsa, bsb, bsc;
  const long* oa;   // per-problem element offsets, else b * bs (the base stays a
  const long* ob;   // kernel argument, so that its loads stay global ones)
  const long* oc;
  int M, N, K;
  double alpha, beta;
  int splits, kchunk;   // split-K: each split covers kchunk of K (multiple of BK)
  double* ws;           // partials [split][batch][M][N] when splits > 1
  int batch;
  const unsigned* amaxA;   // F16 split: largest |A| and |B| as FP32 bits
  const unsigned* amaxB;
  int ws_cm;            // partials [split][batch][N][M] (column-major outputs)
};

__device__ __forceinline__ long off0(const int* t, long s, int i) { return t ? (long)t[i] : (long)i * s; }
template <typename T>
__device__ __forceinline__ T* batch_base(T* p, const long* off, long bs, int b) { return p + (off ? off[b] : (long)b * bs); }

// Raw buffer access to the whole 4 GiB range above `p` (stride 0, no range
// check in effect): the per-lane offset is one 32-bit byte offset, the base a
// scalar descriptor.  Callers keep every offset below 2^32 bytes.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const double* p) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(p), (short)0, -1, 0x00020000);
}
// ... and to the `elems` doubles above `p` only: loads past them return zero
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const double* p, long elems) {
  const long bytes = elems > 0 ? 8 * elems : 0;
  const int n = bytes >= 0xffffffffL ? -1 : (int)(unsigned)bytes;
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(p), (short)0, n, 0x00020000);
}
__device__ __forceinline__ double buffer_load_f64(__amdgpu_buffer_rsrc_t r, unsigned byte_off) {
  typedef unsigned u2 __attribute__((ext_vector_type(2)));
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 0));
}

// Workgroups are dispatched to the 8 XCDs round-robin by linear id; remap so
// that each XCD runs one contiguous range of (tile, split, batch) indices.
// Neighbouring output tiles share rows of A, which then stay in that XCD's L2.
__device__ __forceinline__ void xcd_remap(int& tile, int& split, int& b) {
  const unsigned nx = gridDim.x, ny = gridDim.y;
  const unsigned total = nx * ny * gridDim.z;
  const unsigned lin = blockIdx.x + nx * (blockIdx.y + ny * blockIdx.z);
  const unsigned q = total / 8, r = total % 8, x = lin % 8, i = lin / 8;
  const unsigned id = (x < r) ? x * (q + 1) + i : r * (q + 1) + (x - r) * q + i;
  tile = (int)(id % nx);
  split = (int)((id / nx) % ny);
  b = (int)(id / (nx * ny));
}

// TBL: some operand index goes through an offset table.  Without tables a
// k-tile is loaded from one uniform base per operand plus per-thread 32-bit
// offsets: rows and columns past the edge are clamped to the last valid one
// (their products land in outputs that are not stored), so only a partial
// last k-tile needs a guard, on k.
template <int BM, int BN, int WAVES_M, bool A_KC, bool B_KC, bool TBL>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void gemm_f64_kernel(KArgs g) {
  constexpr int BK = 16;
  constexpr int LDK = BK + 1;
  constexpr int WAVES_N = 4 / WAVES_M;
  constexpr int WM = BM / WAVES_M, WN = BN / WAVES_N;
  constexpr int TM = WM / 16, TN = WN / 16;
  constexpr int EA = BM * BK / 256, EB = BN * BK / 256;
  static_assert(TM >= 1 && TN >= 1 && EA >= 1 && EB >= 1, "tile");
  __shared__ double As[2][BM * LDK];
  __shared__ double Bs[2][BN * LDK];

  // the wave index is uniform: kept scalar, so the per-wave tile offsets take no vector registers
  const int tid = threadIdx.x, lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int tiles_n = (g.N + BN - 1) / BN, tiles_m = (g.M + BM - 1) / BM;
  int tile, split, b;
  xcd_remap(tile, split, b);
  // consecutive tiles share the larger operand's block (A rows or B columns)
  const bool mfast = g.N > g.M;
  const int tm_ = mfast ? tile % tiles_m : tile / tiles_n;
  const int tn_ = mfast ? tile / tiles_m : tile % tiles_n;
  const int m0 = tm_ * BM, n0 = tn_ * BN;
  const int kb = split * g.kchunk;
  const int ke = min(g.K, kb + g.kchunk);
  const double* A = batch_base(g.A, g.oa, g.bsa, b);
  const double* B = batch_base(g.B, g.ob, g.bsb, b);

  // ---- per-thread load coordinates ------------------------------------
  // A tile element (r, kk): A_KC -> threads walk k fastest, else m fastest.
  int a_r[EA], a_k[EA];
  long a_roff[EA];
  bool a_rok[EA];
#pragma unroll
  for (int j = 0; j < EA; ++j) {
    int e = tid + 256 * j;
    if (A_KC) { a_k[j] = e % BK; a_r[j] = e / BK; }
    else      { a_r[j] = e % BM; a_k[j] = e / BM; }
    int m = m0 + a_r[j];
    a_rok[j] = m < g.M;
    a_roff[j] = a_rok[j] ? off0(g.ta0, g.sa0, m) : 0;
  }
  int b_c[EB], b_k[EB];
  long b_coff[EB];
  bool b_cok[EB];
#pragma unroll
  for (int j = 0; j < EB; ++j) {
    int e = tid + 256 * j;
    if (B_KC) { b_k[j] = e % BK; b_c[j] = e / BK; }
    else      { b_c[j] = e % BN; b_k[j] = e / BN; }
    int n = n0 + b_c[j];
    b_cok[j] = n < g.N;
    b_coff[j] = b_cok[j] ? off0(g.tb1, g.sb1, n) : 0;
  }
  // table-free offsets within a k-tile (edge rows / columns clamped)
  // (byte offsets for buffer loads: one 32-bit register per load, no 64-bit
  // address arithmetic)
  unsigned a_off[EA], b_off[EB];
  if (!TBL) {
#pragma unroll
    for (int j = 0; j < EA; ++j)
      a_off[j] = 8u * (unsigned)((long)min(m0 + a_r[j], g.M - 1) * g.sa0 + (long)a_k[j] * g.sa1);
#pragma unroll
    for (int j = 0; j < EB; ++j)
      b_off[j] = 8u * (unsigned)((long)min(n0 + b_c[j], g.N - 1) * g.sb1 + (long)b_k[j] * g.sb0);
  }
  // one past the last element of each operand, in elements from its base
  const long a_end = (long)(g.M - 1) * g.sa0 + (long)(g.K - 1) * g.sa1 + 1;
  const long b_end = (long)(g.N - 1) * g.sb1 + (long)(g.K - 1) * g.sb0 + 1;

  // Two register sets for k-tiles in flight: while the MFMAs run on one LDS
  // buffer, one set is stored to the other buffer and the other set receives
  // the loads of the tile after it.  The sets alternate from one k-tile to
  // the next (the loop is unrolled by two), so a tile's loads have a whole
  // k-step before their registers are stored, and no register copies.
  // Without tables every k-step issues the same eight loads (the last steps
  // reload the last tile; loads past an operand's end return zero), so the
  // waits before the stores count exactly the older set; the slots of a
  // partial last tile at k >= ke are zeroed when it is stored.
  // With tables (their offsets take the registers) only the first set is used.
  double ra[EA], rb[EB], ra2[EA], rb2[EB];
  auto load_tile = [&](int k0, double (&xa)[EA], double (&xb)[EB]) {
    if (!TBL) {
      const __amdgpu_buffer_rsrc_t Ak = buffer_rsrc(A + (long)k0 * g.sa1, a_end - (long)k0 * g.sa1);
      const __amdgpu_buffer_rsrc_t Bk = buffer_rsrc(B + (long)k0 * g.sb0, b_end - (long)k0 * g.sb0);
#pragma unroll
      for (int j = 0; j < EA; ++j) xa[j] = buffer_load_f64(Ak, a_off[j]);
#pragma unroll
      for (int j = 0; j < EB; ++j) xb[j] = buffer_load_f64(Bk, b_off[j]);
      return;
    }
#pragma unroll
    for (int j = 0; j < EA; ++j) {
      int k = k0 + a_k[j];
      xa[j] = (a_rok[j] && k < ke) ? A[a_roff[j] + off0(g.ta1, g.sa1, k)] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < EB; ++j) {
      int k = k0 + b_k[j];
      xb[j] = (b_cok[j] && k < ke) ? B[b_coff[j] + off0(g.tb0, g.sb0, k)] : 0.0;
    }
  };
  // LDS slot of each staged element: where the 256-thread step of the load
  // pattern is a whole number of rows (k walked fastest) or of k columns, the
  // slots of one lane are one base plus constant steps (immediate offsets).
  constexpr bool A_LIN = A_KC ? (256 % BK == 0) : (256 % BM == 0);
  constexpr bool B_LIN = B_KC ? (256 % BK == 0) : (256 % BN == 0);
  constexpr int A_JS = A_KC ? (256 / BK) * LDK : 256 / BM;
  constexpr int B_JS = B_KC ? (256 / BK) * LDK : 256 / BN;
  const int a_st = a_r[0] * LDK + a_k[0], b_st = b_c[0] * LDK + b_k[0];
  auto a_slot = [&](int j) { return A_LIN ? a_st + j * A_JS : a_r[j] * LDK + a_k[j]; };
  auto b_slot = [&](int j) { return B_LIN ? b_st + j * B_JS : b_c[j] * LDK + b_k[j]; };
  auto store_tile = [&](int buf, const double (&xa)[EA], const double (&xb)[EB]) {
#pragma unroll
    for (int j = 0; j < EA; ++j) As[buf][a_slot(j)] = xa[j];
#pragma unroll
    for (int j = 0; j < EB; ++j) Bs[buf][b_slot(j)] = xb[j];
  };
  // table-free tiles: the tile starting at k0 may be partial
  auto store_tile_k = [&](int buf, int k0, const double (&xa)[EA], const double (&xb)[EB]) {
    if (k0 + BK <= ke) {
      store_tile(buf, xa, xb);
      return;
    }
#pragma unroll
    for (int j = 0; j < EA; ++j) As[buf][a_slot(j)] = (k0 + a_k[j] < ke) ? xa[j] : 0.0;
#pragma unroll
    for (int j = 0; j < EB; ++j) Bs[buf][b_slot(j)] = (k0 + b_k[j] < ke) ? xb[j] : 0.0;
  };

  d4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};

  const int wm0 = (wave / WAVES_N) * WM, wn0 = (wave % WAVES_N) * WN;
  const int r16 = lane & 15, kg = lane >> 4;

  // one k-tile of MFMAs from LDS buffer `cur`; fragments loaded per k-slot,
  // next to their MFMAs (fewer live registers)
  auto compute = [&](int cur) {
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      double af[TM], bf[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) af[i] = As[cur][(wm0 + i * 16 + r16) * LDK + 4 * kg + s];
#pragma unroll
      for (int j = 0; j < TN; ++j) bf[j] = Bs[cur][(wn0 + j * 16 + r16) * LDK + 4 * kg + s];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(af[i], bf[j], acc[i][j], 0, 0, 0);
    }
  };

  const int nk = (ke > kb) ? (ke - kb + BK - 1) / BK : 0;
  if (TBL) {
    if (nk > 0) {
      load_tile(kb, ra, rb);
      store_tile(0, ra, rb);
    }
    __syncthreads();
    for (int it = 0; it < nk; ++it) {
      const int cur = it & 1;
      if (it + 1 < nk) load_tile(kb + (it + 1) * BK, ra, rb);
      compute(cur);
      if (it + 1 < nk) store_tile(cur ^ 1, ra, rb);
      __syncthreads();
    }
  } else if (nk > 0) {
    // even k-tiles: loads into set 2 while set 1 (the next tile) is stored;
    // odd k-tiles: the other way round
    const int last = kb + (nk - 1) * BK;
    auto kt = [&](int t) { return min(kb + t * BK, last); };
    load_tile(kb, ra2, rb2);
    store_tile_k(0, kb, ra2, rb2);
    load_tile(kt(1), ra, rb);
    __syncthreads();
    for (int it = 0; it < nk; it += 2) {
      load_tile(kt(it + 2), ra2, rb2);
      compute(0);
      if (it + 1 < nk) store_tile_k(1, kt(it + 1), ra, rb);
      __syncthreads();
      if (it + 1 >= nk) break;
      load_tile(kt(it + 3), ra, rb);
      compute(1);
      if (it + 2 < nk) store_tile_k(0, kt(it + 2), ra2, rb2);
      __syncthreads();
    }
  }

  // ---- epilogue ----------------------------------------------------------
  double* C = batch_base(g.C, g.oc, g.bsc, b);
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int m = m0 + wm0 + i * 16 + kg + 4 * r;
        int n = n0 + wn0 + j * 16 + r16;
        if (m < g.M && n < g.N) {
          double v = g.alpha * acc[i][j][r];
          if (g.splits > 1) {
            g.ws[(((long)split * g.batch + b) * g.M + m) * g.N + n] = v;
          } else {
            long o = off0(g.tc0, g.sc0, m) + off0(g.tc1, g.sc1, n);
            C[o] = (g.beta == 0.0) ? v : v + g.beta * C[o];
          }
        }
      }
}

// Sum the split-K partials in split order (deterministic) into C.
// With ws_cm the partials and the walk run m fastest, so that a column-major
// C is written along its columns.
__global__ void splitk_reduce(KArgs g) {
  long total = (long)g.batch * g.M * g.N;
  for (long e = blockIdx.x * (long)blockDim.x + threadIdx.x; e < total; e += (long)gridDim.x * blockDim.x) {
    int m, n, b;
    if (g.ws_cm) {
      m = (int)(e % g.M);
      const long t = e / g.M;
      n = (int)(t % g.N);
      b = (int)(t / g.N);
    } else {
      n = (int)(e % g.N);
      const long t = e / g.N;
      m = (int)(t % g.M);
      b = (int)(t / g.M);
    }
    double s = 0.0;
    for (int k = 0; k < g.splits; ++k)
      s += g.ws_cm ? g.ws[(((long)k * g.batch + b) * g.N + n) * g.M + m]
                   : g.ws[(((long)k * g.batch + b) * g.M + m) * g.N + n];
    double* C = batch_base(g.C, g.oc, g.bsc, b);
    long o = off0(g.tc0, g.sc0, m) + off0(g.tc1, g.sc1, n);
    C[o] = (g.beta == 0.0) ? s : s + g.beta * C[o];
  }
}

template <int BM, int BN, int WAVES_M, bool TBL>
void launch_f64_t(hipStream_t st, const KArgs& g, bool a_kc, bool b_kc, dim3 grid) {
  if (a_kc && b_kc)
    hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, WAVES_M, true, true, TBL>), grid, dim3(256), 0, st, g);
  else if (a_kc && !b_kc)
    hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, WAVES_M, true, false, TBL>), grid, dim3(256), 0, st, g);
  else if (!a_kc && b_kc)
    hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, WAVES_M, false, true, TBL>), grid, dim3(256), 0, st, g);
  else
    hipLaunchKernelGGL((gemm_f64_kernel<BM, BN, WAVES_M, false, false, TBL>), grid, dim3(256), 0, st, g);
}

// The table-free kernels take 32-bit byte offsets within a tile (k-tiles of
// at most 32): elements below 2^29.
bool needs_tables(const KArgs& g, long kMaxOff) {
  return g.ta0 || g.ta1 || g.tb0 || g.tb1 || g.sa0 < 0 || g.sa1 < 0 || g.sb0 < 0 || g.sb1 < 0 ||
         (long)g.M * g.sa0 + 32L * g.sa1 > kMaxOff || (long)g.N * g.sb1 + 32L * g.sb0 > kMaxOff;
}

template <int BM, int BN, int WAVES_M>
void launch_f64(hipStream_t st, const KArgs& g, bool a_kc, bool b_kc, dim3 grid) {
  if (needs_tables(g, 0x1fffffffL)) launch_f64_t<BM, BN, WAVES_M, true>(st, g, a_kc, b_kc, grid);
  else                 launch_f64_t<BM, BN, WAVES_M, false>(st, g, a_kc, b_kc, grid);
}

// ---------------------------------------------------------------------------
// Reduced-precision kernels: FP64 operands are rounded while being staged into
// LDS (k contiguous per row, padded so that every lane's 8-element fragment
// is one 16-byte LDS read and the 16 rows of a fragment hit distinct banks);
// MFMA with FP32 accumulation; the epilogue widens to FP64.
//
// Lane layouts (checked on gfx950 against exact integer products):
//   v_mfma_f32_16x16x4f32:          lane l supplies A[l%16][k(l/16)], B[k(l/16)][l%16];
//   v_mfma_f32_16x16x32_{bf16,f16}: lane l supplies A[l%16][8(l/16)+i], B[8(l/16)+i][l%16], i < 8;
//   both return D[4(l/16)+r][l%16] in register r.
// In the FP32 kernel the eight MFMAs of a 32-wide K step take k = 8(l/16)+s
// at step s, so each lane also reads eight contiguous values.
// ---------------------------------------------------------------------------
typedef float f4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 h8 __attribute__((ext_vector_type(8)));

enum { LP_F32 = 1, LP_BF16 = 2, LP_F16 = 3 };

template <int KIND> struct LpStore;
template <> struct LpStore<LP_F32> { typedef float T; };
template <> struct LpStore<LP_BF16> { typedef __bf16 T; };
template <> struct LpStore<LP_F16> { typedef _Float16 T; };

// 2^s with |x| * 2^s <= 2^14 for every entry x of an operand whose largest
// magnitude is m (FP32 bits); 1 for m = 0 or non-finite m.
__device__ __forceinline__ double f16_scale(unsigned mbits) {
  const float m = __uint_as_float(mbits);
  if (!(m > 0.0f) || !(m < 3.0e38f)) return 1.0;
  return ldexp(1.0, 14 - (ilogbf(m) + 1));
}

template <int KIND, int BM, int BN, int WAVES_M, bool A_KC, bool B_KC, bool TBL>
__global__ __launch_bounds__(256) void gemm_lp_kernel(KArgs g) {
  typedef typename LpStore<KIND>::T T;
  constexpr int BK = 32;
  constexpr int LDK = BK + (KIND == LP_F32 ? 4 : 8);
  constexpr int NP = (KIND == LP_F16) ? 2 : 1;   // hi (and lo) parts
  constexpr int WAVES_N = 4 / WAVES_M;
  constexpr int WM = BM / WAVES_M, WN = BN / WAVES_N;
  constexpr int TM = WM / 16, TN = WN / 16;
  constexpr int EA = BM * BK / 256, EB = BN * BK / 256;
  constexpr bool PAIRS = KIND == LP_BF16;
  static_assert(TM >= 1 && TN >= 1 && EA >= 2 && EB >= 2 && EA % 2 == 0 && EB % 2 == 0, "tile (pairs of k)");
  __shared__ __attribute__((aligned(16))) T As[2][NP][BM * LDK];
  __shared__ __attribute__((aligned(16))) T Bs[2][NP][BN * LDK];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tiles_n = (g.N + BN - 1) / BN, tiles_m = (g.M + BM - 1) / BM;
  int tile, split, b;
  xcd_remap(tile, split, b);
  // consecutive tiles share the larger operand's block (A rows or B columns)
  const bool mfast = g.N > g.M;
  const int tm_ = mfast ? tile % tiles_m : tile / tiles_n;
  const int tn_ = mfast ? tile / tiles_m : tile % tiles_n;
  const int m0 = tm_ * BM, n0 = tn_ * BN;
  const int kb = split * g.kchunk;
  const int ke = min(g.K, kb + g.kchunk);
  const double* A = batch_base(g.A, g.oa, g.bsa, b);
  const double* B = batch_base(g.B, g.ob, g.bsb, b);
  double sa = 1.0, sb = 1.0;
  if (KIND == LP_F16) {
    sa = f16_scale(*g.amaxA);
    sb = f16_scale(*g.amaxB);
  }

  int a_r[EA], a_k[EA];
  long a_roff[EA];
  bool a_rok[EA];
#pragma unroll
  for (int j = 0; j < EA; ++j) {
    // BF16 with k contiguous: each thread takes pairs of consecutive k of one
    // row (one packed LDS store per pair); else k (A_KC) or m walked fastest
    if (A_KC && PAIRS) {
      const int e = tid + 256 * (j / 2);
      a_k[j] = (e % (BK / 2)) * 2 + (j & 1);
      a_r[j] = e / (BK / 2);
    } else {
      const int e = tid + 256 * j;
      if (A_KC) { a_k[j] = e % BK; a_r[j] = e / BK; }
      else      { a_r[j] = e % BM; a_k[j] = e / BM; }
    }
    int m = m0 + a_r[j];
    a_rok[j] = m < g.M;
    a_roff[j] = a_rok[j] ? off0(g.ta0, g.sa0, m) : 0;
  }
  int b_c[EB], b_k[EB];
  long b_coff[EB];
  bool b_cok[EB];
#pragma unroll
  for (int j = 0; j < EB; ++j) {
    if (B_KC && PAIRS) {
      const int e = tid + 256 * (j / 2);
      b_k[j] = (e % (BK / 2)) * 2 + (j & 1);
      b_c[j] = e / (BK / 2);
    } else {
      const int e = tid + 256 * j;
      if (B_KC) { b_k[j] = e % BK; b_c[j] = e / BK; }
      else      { b_c[j] = e % BN; b_k[j] = e / BN; }
    }
    int n = n0 + b_c[j];
    b_cok[j] = n < g.N;
    b_coff[j] = b_cok[j] ? off0(g.tb1, g.sb1, n) : 0;
  }
  // table-free byte offsets within a k-tile (edge rows / columns clamped) for
  // buffer loads, as in the FP64 kernel
  unsigned a_off[EA], b_off[EB];
  if (!TBL) {
#pragma unroll
    for (int j = 0; j < EA; ++j)
      a_off[j] = 8u * (unsigned)((long)min(m0 + a_r[j], g.M - 1) * g.sa0 + (long)a_k[j] * g.sa1);
#pragma unroll
    for (int j = 0; j < EB; ++j)
      b_off[j] = 8u * (unsigned)((long)min(n0 + b_c[j], g.N - 1) * g.sb1 + (long)b_k[j] * g.sb0);
  }
  const long a_end = (long)(g.M - 1) * g.sa0 + (long)(g.K - 1) * g.sa1 + 1;
  const long b_end = (long)(g.N - 1) * g.sb1 + (long)(g.K - 1) * g.sb0 + 1;

  // Without tables FP32 keeps two register sets of loads that alternate from
  // one k-tile to the next, as the FP64 kernel does; BF16 (the second set
  // costs it a wave per SIMD), split FP16 (two operand parts in LDS) and the
  // table-addressed loads use one set, loaded one k-tile ahead.
  constexpr bool PF2 = !TBL && KIND == LP_F32;
  double ra[EA], rb[EB], ra2[EA], rb2[EB];
  auto load_tile = [&](int k0, double (&xa)[EA], double (&xb)[EB]) {
    if (!TBL) {
      const __amdgpu_buffer_rsrc_t Ak = buffer_rsrc(A + (long)k0 * g.sa1, a_end - (long)k0 * g.sa1);
      const __amdgpu_buffer_rsrc_t Bk = buffer_rsrc(B + (long)k0 * g.sb0, b_end - (long)k0 * g.sb0);
#pragma unroll
      for (int j = 0; j < EA; ++j) xa[j] = buffer_load_f64(Ak, a_off[j]);
#pragma unroll
      for (int j = 0; j < EB; ++j) xb[j] = buffer_load_f64(Bk, b_off[j]);
      return;
    }
#pragma unroll
    for (int j = 0; j < EA; ++j) {
      int k = k0 + a_k[j];
      xa[j] = (a_rok[j] && k < ke) ? A[a_roff[j] + off0(g.ta1, g.sa1, k)] : 0.0;
    }
#pragma unroll
    for (int j = 0; j < EB; ++j) {
      int k = k0 + b_k[j];
      xb[j] = (b_cok[j] && k < ke) ? B[b_coff[j] + off0(g.tb0, g.sb0, k)] : 0.0;
    }
  };
  auto put = [&](T* hi, T* lo, int idx, double x, double sc) {
    if constexpr (KIND == LP_F16) {
      const double xs = x * sc;                        // exact (power of two)
      const _Float16 h = (_Float16)(float)xs;
      hi[idx] = h;
      lo[idx] = (_Float16)(float)((xs - (double)h) * 2048.0);
    } else {
      hi[idx] = (T)(float)x;
    }
  };
  // two consecutive-k values of one row -> LDS as one packed store
  auto put2 = [&](T* hi, T* lo, int idx, double x0, double x1, double sc) {
    typedef T t2 __attribute__((ext_vector_type(2)));
    if constexpr (KIND == LP_F16) {
      const double y0 = x0 * sc, y1 = x1 * sc;           // exact (power of two)
      const _Float16 h0 = (_Float16)(float)y0, h1 = (_Float16)(float)y1;
      *reinterpret_cast<t2*>(hi + idx) = t2{h0, h1};
      *reinterpret_cast<t2*>(lo + idx) =
          t2{(_Float16)(float)((y0 - (double)h0) * 2048.0), (_Float16)(float)((y1 - (double)h1) * 2048.0)};
    } else {
      *reinterpret_cast<t2*>(hi + idx) = t2{(T)(float)x0, (T)(float)x1};
    }
  };
  // store the tile starting at k0; the slots of a partial tile at k >= ke
  // are zeroed (a separate path, so that whole tiles take no selects)
  auto store_body = [&](int buf, int k0, const double (&xa)[EA], const double (&xb)[EB], auto part_tag) {
    constexpr bool part = decltype(part_tag)::value;
    if constexpr (A_KC && PAIRS) {
#pragma unroll
      for (int j = 0; j < EA; j += 2) {
        const double x0 = (!part || k0 + a_k[j] < ke) ? xa[j] : 0.0;
        const double x1 = (!part || k0 + a_k[j + 1] < ke) ? xa[j + 1] : 0.0;
        put2(As[buf][0], As[buf][NP - 1], a_r[j] * LDK + a_k[j], x0, x1, sa);
      }
    } else {
#pragma unroll
      for (int j = 0; j < EA; ++j)
        put(As[buf][0], As[buf][NP - 1], a_r[j] * LDK + a_k[j], (!part || k0 + a_k[j] < ke) ? xa[j] : 0.0, sa);
    }
    if constexpr (B_KC && PAIRS) {
#pragma unroll
      for (int j = 0; j < EB; j += 2) {
        const double x0 = (!part || k0 + b_k[j] < ke) ? xb[j] : 0.0;
        const double x1 = (!part || k0 + b_k[j + 1] < ke) ? xb[j + 1] : 0.0;
        put2(Bs[buf][0], Bs[buf][NP - 1], b_c[j] * LDK + b_k[j], x0, x1, sb);
      }
    } else {
#pragma unroll
      for (int j = 0; j < EB; ++j)
        put(Bs[buf][0], Bs[buf][NP - 1], b_c[j] * LDK + b_k[j], (!part || k0 + b_k[j] < ke) ? xb[j] : 0.0, sb);
    }
  };
  // (BF16 measured 2.5% faster over the sweep with the masked path for every
  // tile, FP32 and split FP16 2% slower)
  auto store_tile = [&](int buf, int k0, const double (&xa)[EA], const double (&xb)[EB]) {
    if (KIND != LP_BF16 && k0 + BK <= ke)
      store_body(buf, k0, xa, xb, std::false_type{});
    else
      store_body(buf, k0, xa, xb, std::true_type{});
  };

  f4 acc[TM][TN], acc2[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      acc2[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    }

  const int wm0 = (wave / WAVES_N) * WM, wn0 = (wave % WAVES_N) * WN;
  const int r16 = lane & 15, kg = lane >> 4;

  // one k-tile of MFMAs from LDS buffer `cur`
  auto compute = [&](int cur) {
    if constexpr (KIND == LP_F32) {
      f4 af[TM][2], bfr[TN][2];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const f4* p = reinterpret_cast<const f4*>(&As[cur][0][(wm0 + i * 16 + r16) * LDK + 8 * kg]);
        af[i][0] = p[0];
        af[i][1] = p[1];
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const f4* p = reinterpret_cast<const f4*>(&Bs[cur][0][(wn0 + j * 16 + r16) * LDK + 8 * kg]);
        bfr[j][0] = p[0];
        bfr[j][1] = p[1];
      }
#pragma unroll
      for (int s = 0; s < 8; ++s)
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(af[i][s >> 2][s & 3], bfr[j][s >> 2][s & 3],
                                                             acc[i][j], 0, 0, 0);
    } else if constexpr (KIND == LP_BF16) {
      bf8 af[TM], bfr[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i)
        af[i] = *reinterpret_cast<const bf8*>(&As[cur][0][(wm0 + i * 16 + r16) * LDK + 8 * kg]);
#pragma unroll
      for (int j = 0; j < TN; ++j)
        bfr[j] = *reinterpret_cast<const bf8*>(&Bs[cur][0][(wn0 + j * 16 + r16) * LDK + 8 * kg]);
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
    } else {
      h8 ah[TM], al[TM], bh[TN], bl[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int o = (wm0 + i * 16 + r16) * LDK + 8 * kg;
        ah[i] = *reinterpret_cast<const h8*>(&As[cur][0][o]);
        al[i] = *reinterpret_cast<const h8*>(&As[cur][NP - 1][o]);
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int o = (wn0 + j * 16 + r16) * LDK + 8 * kg;
        bh[j] = *reinterpret_cast<const h8*>(&Bs[cur][0][o]);
        bl[j] = *reinterpret_cast<const h8*>(&Bs[cur][NP - 1][o]);
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[i], bh[j], acc[i][j], 0, 0, 0);
          acc2[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[i], bl[j], acc2[i][j], 0, 0, 0);
          acc2[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[i], bh[j], acc2[i][j], 0, 0, 0);
        }
    }
  };

  const int nk = (ke > kb) ? (ke - kb + BK - 1) / BK : 0;
  if (PF2) {
    if (nk > 0) {
      // even k-tiles: loads into set 2 while set 1 (the next tile) is
      // stored; odd k-tiles the other way round; the last steps reload the
      // last tile so that every step issues the same loads
      const int last = kb + (nk - 1) * BK;
      auto kt = [&](int t) { return min(kb + t * BK, last); };
      load_tile(kb, ra2, rb2);
      store_tile(0, kb, ra2, rb2);
      load_tile(kt(1), ra, rb);
      __syncthreads();
      for (int it = 0; it < nk; it += 2) {
        load_tile(kt(it + 2), ra2, rb2);
        compute(0);
        if (it + 1 < nk) store_tile(1, kt(it + 1), ra, rb);
        __syncthreads();
        if (it + 1 >= nk) break;
        load_tile(kt(it + 3), ra, rb);
        compute(1);
        if (it + 2 < nk) store_tile(0, kt(it + 2), ra2, rb2);
        __syncthreads();
      }
    }
  } else {
    if (nk > 0) {
      load_tile(kb, ra, rb);
      store_tile(0, kb, ra, rb);
    }
    __syncthreads();
    for (int it = 0; it < nk; ++it) {
      const int cur = it & 1;
      if (it + 1 < nk) load_tile(kb + (it + 1) * BK, ra, rb);
      compute(cur);
      if (it + 1 < nk) store_tile(cur ^ 1, kb + (it + 1) * BK, ra, rb);
      __syncthreads();
    }
  }

  double* C = batch_base(g.C, g.oc, g.bsc, b);
  const double unscale = g.alpha / (sa * sb);
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        int m = m0 + wm0 + i * 16 + kg * 4 + r;
        int n = n0 + wn0 + j * 16 + r16;
        if (m < g.M && n < g.N) {
          double v = (double)acc[i][j][r];
          if constexpr (KIND == LP_F16) v += (double)acc2[i][j][r] * (1.0 / 2048.0);
          v *= unscale;
          if (g.splits > 1) {
            g.ws[(((long)split * g.batch + b) * g.M + m) * g.N + n] = v;
          } else {
            long o = off0(g.tc0, g.sc0, m) + off0(g.tc1, g.sc1, n);
            C[o] = (g.beta == 0.0) ? v : v + g.beta * C[o];
          }
        }
      }
}

// ---------------------------------------------------------------------------
// Products of pre-converted operands (PreOperand): both operands are 2-byte
// values with k contiguous and whole 32-wide k-tiles, so a lane stages eight
// values of one row with one 16-byte load and one 16-byte LDS store, with no
// conversion and no k guard; rows past M (N) are clamped to the last one
// (their products are not stored).  Same LDS layout, MFMA lane layout and
// epilogue as gemm_lp_kernel.
// ---------------------------------------------------------------------------
struct PArgs {
  const unsigned short* A;
  const unsigned short* B;
  double* C;
  long lda, bsa, loa, ldb, bsb, lob;
  long sc0, sc1, bsc;
  int M, N, Kp;
  double alpha;
  const unsigned* amaxA;
  const unsigned* amaxB;
  const float* rsA;
  const float* rsB;
  long rsa_bs, rsb_bs;
  int splits, kchunk;
  double* ws;
  int batch;
  int ws_cm;   // partials [split][batch][N][M] (column-major C)
};

template <int KIND, int BM, int BN, int WAVES_M, int WAVES_N, int STAGES>
__global__ __launch_bounds__(64 * WAVES_M * WAVES_N) void gemm_pre_kernel(PArgs g) {
  typedef typename LpStore<KIND>::T T;
  typedef unsigned int u4 __attribute__((ext_vector_type(4)));
  constexpr int NT = 64 * WAVES_M * WAVES_N;
  // LDS rows of 32 values (four 16-byte chunks) without padding; chunk q of
  // row r sits at position q ^ ((r >> 1) & 3), so that the eight lanes of a
  // 16-byte store phase (two rows, four chunks each) and of a fragment read
  // phase (eight rows, one chunk) hit eight distinct bank quads
  constexpr int BK = 32, LDK = BK;
  constexpr int NP = (KIND == LP_F16) ? 2 : 1;
  constexpr int WM = BM / WAVES_M, WN = BN / WAVES_N;
  constexpr int TM = WM / 16, TN = WN / 16;
  // 16-byte chunks (eight k values of a row) per thread and k-tile; the last
  // round of a count that is not a multiple of the threads is guarded
  constexpr int NCA = BM * (BK / 8), NCB = BN * (BK / 8);
  constexpr int CA = (NCA + NT - 1) / NT, CB = (NCB + NT - 1) / NT;
  static_assert(TM >= 1 && TN >= 1 && WM % 16 == 0 && WN % 16 == 0, "tile");
  __shared__ __attribute__((aligned(16))) T As[2][NP][BM * LDK];
  __shared__ __attribute__((aligned(16))) T Bs[2][NP][BN * LDK];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int tiles_n = (g.N + BN - 1) / BN, tiles_m = (g.M + BM - 1) / BM;
  int tile, split, b;
  xcd_remap(tile, split, b);
  // consecutive tiles walk the rows of A (the large operand) in order
  const int tm_ = tile % tiles_m, tn_ = tile / tiles_m;
  (void)tiles_n;
  const int m0 = tm_ * BM, n0 = tn_ * BN;
  const int kb = split * g.kchunk;
  const int ke = min(g.Kp, kb + g.kchunk);
  const unsigned short* A = g.A + (long)b * g.bsa;
  const unsigned short* B = g.B + (long)b * g.bsb;

  long a_off[CA], b_off[CB];
  int a_lds[CA], b_lds[CB];
  bool a_in[CA], b_in[CB];
#pragma unroll
  for (int j = 0; j < CA; ++j) {
    const int e = tid + NT * j, r = e / (BK / 8), kq = (e % (BK / 8)) * 8;
    a_in[j] = (NCA % NT == 0) || e < NCA;
    a_off[j] = (long)min(m0 + (a_in[j] ? r : 0), g.M - 1) * g.lda + kq;
    a_lds[j] = a_in[j] ? r * LDK + ((kq >> 3) ^ ((r >> 1) & 3)) * 8 : 0;
  }
#pragma unroll
  for (int j = 0; j < CB; ++j) {
    const int e = tid + NT * j, r = e / (BK / 8), kq = (e % (BK / 8)) * 8;
    b_in[j] = (NCB % NT == 0) || e < NCB;
    b_off[j] = (long)min(n0 + (b_in[j] ? r : 0), g.N - 1) * g.ldb + kq;
    b_lds[j] = b_in[j] ? r * LDK + ((kq >> 3) ^ ((r >> 1) & 3)) * 8 : 0;
  }
  // STAGES k-tiles in flight in registers (the loads of tile t + STAGES are
  // issued when tile t + 1 moves to LDS), so that a k-tile's global load
  // latency is spread over several tiles of MFMAs
  u4 ra[STAGES][NP][CA], rb[STAGES][NP][CB];
  auto load_tile = [&](int st, int k0) {
#pragma unroll
    for (int p = 0; p < NP; ++p) {
#pragma unroll
      for (int j = 0; j < CA; ++j)   // unconditional (a_off of an unused chunk is a valid row): uniform counts
        ra[st][p][j] = *reinterpret_cast<const u4*>(A + (p ? g.loa : 0) + a_off[j] + k0);
#pragma unroll
      for (int j = 0; j < CB; ++j)
        rb[st][p][j] = *reinterpret_cast<const u4*>(B + (p ? g.lob : 0) + b_off[j] + k0);
    }
  };
  auto store_tile = [&](int st, int buf) {
#pragma unroll
    for (int p = 0; p < NP; ++p) {
#pragma unroll
      for (int j = 0; j < CA; ++j)
        if (a_in[j]) *reinterpret_cast<u4*>(&As[buf][p][a_lds[j]]) = ra[st][p][j];
#pragma unroll
      for (int j = 0; j < CB; ++j)
        if (b_in[j]) *reinterpret_cast<u4*>(&Bs[buf][p][b_lds[j]]) = rb[st][p][j];
    }
  };

  f4 acc[TM][TN], acc2[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
      acc2[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    }
  const int wm0 = (wave / WAVES_N) * WM, wn0 = (wave % WAVES_N) * WN;
  const int r16 = lane & 15, kg = lane >> 4;
  // position of this lane's fragment (chunk kg) in LDS row `row`
  auto frag = [&](int row) { return row * LDK + ((kg ^ ((row >> 1) & 3)) * 8); };
  auto compute = [&](int cur) {
    if constexpr (KIND == LP_BF16) {
      bf8 af[TM], bfr[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) af[i] = *reinterpret_cast<const bf8*>(&As[cur][0][frag(wm0 + i * 16 + r16)]);
#pragma unroll
      for (int j = 0; j < TN; ++j) bfr[j] = *reinterpret_cast<const bf8*>(&Bs[cur][0][frag(wn0 + j * 16 + r16)]);
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[i], bfr[j], acc[i][j], 0, 0, 0);
    } else {
      h8 ah[TM], al[TM], bh[TN], bl[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int o = frag(wm0 + i * 16 + r16);
        ah[i] = *reinterpret_cast<const h8*>(&As[cur][0][o]);
        al[i] = *reinterpret_cast<const h8*>(&As[cur][NP - 1][o]);
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int o = frag(wn0 + j * 16 + r16);
        bh[j] = *reinterpret_cast<const h8*>(&Bs[cur][0][o]);
        bl[j] = *reinterpret_cast<const h8*>(&Bs[cur][NP - 1][o]);
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[i], bh[j], acc[i][j], 0, 0, 0);
          acc2[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah[i], bl[j], acc2[i][j], 0, 0, 0);
          acc2[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al[i], bh[j], acc2[i][j], 0, 0, 0);
        }
    }
  };

  const int nk = (ke > kb) ? (ke - kb) / BK : 0;
  // Tile t sits in register stage t % STAGES until it moves to LDS buffer
  // t % 2.  Every step of the main loop issues the same loads (tiles past
  // the last one reload the last, and are stored into a buffer no step
  // reads), so that the waits before each store count exactly the younger
  // stages' loads and STAGES tiles stay in flight.
  if (nk > 0) {
    const int last = nk - 1;
    load_tile(0, kb);
    store_tile(0, 0);
#pragma unroll
    for (int t = 1; t <= STAGES; ++t) load_tile(t % STAGES, kb + min(t, last) * BK);
    __syncthreads();
    int it0 = 0;
    for (; it0 + STAGES <= nk; it0 += STAGES) {
#pragma unroll
      for (int u = 0; u < STAGES; ++u) {
        const int it = it0 + u;
        compute(it & 1);
        store_tile((u + 1) % STAGES, (it + 1) & 1);
        load_tile((u + 1) % STAGES, kb + min(it + 1 + STAGES, last) * BK);
        __syncthreads();
      }
    }
#pragma unroll
    for (int u = 0; u < STAGES; ++u) {   // the last nk mod STAGES tiles
      const int it = it0 + u;
      if (it < nk) {
        compute(it & 1);
        if (it + 1 < nk) store_tile((u + 1) % STAGES, (it + 1) & 1);
        __syncthreads();
      }
    }
  }

  // scales: F16 A by one power of two (or one per row), B by one per row
  // of B (column of C); BF16 none
  double sa = 1.0;
  if (KIND == LP_F16 && !g.rsA) sa = f16_scale(*g.amaxA);
  double* C = g.C + (long)b * g.bsc;
#pragma unroll
  for (int j = 0; j < TN; ++j) {
    const int n = n0 + wn0 + j * 16 + r16;
    double sbn = 1.0;
    if (KIND == LP_F16 && n < g.N) sbn = g.rsB ? (double)g.rsB[(long)b * g.rsb_bs + n] : f16_scale(*g.amaxB);
#pragma unroll
    for (int i = 0; i < TM; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm0 + i * 16 + kg * 4 + r;
        if (m < g.M && n < g.N) {
          double v = (double)acc[i][j][r];
          if constexpr (KIND == LP_F16) {
            v += (double)acc2[i][j][r] * (1.0 / 2048.0);
            const double sam = g.rsA ? (double)g.rsA[(long)b * g.rsa_bs + m] : sa;
            v *= g.alpha / (sam * sbn);
          } else {
            v *= g.alpha;
          }
          if (g.splits > 1)
            g.ws[g.ws_cm ? (((long)split * g.batch + b) * g.N + n) * g.M + m
                         : (((long)split * g.batch + b) * g.M + m) * g.N + n] = v;
          else
            C[m * g.sc0 + n * g.sc1] = v;
        }
      }
  }
}

// Square operand -> pre-converted rows of G and of G^T: 32 x 32 tiles through
// LDS, so that both outputs are written along their rows.  Values past n
// (the padding up to ld) are written as zeros.
template <int KIND>
__global__ __launch_bounds__(256) void k_convert_square_pre(const double* G, long gbs, int n, long ld,
                                                            unsigned short* out, long obs, long lo,
                                                            const unsigned* amax) {
  typedef typename LpStore<KIND>::T T;
  __shared__ double t[32][33];
  const int b = blockIdx.z, r0 = blockIdx.y * 32, c0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  const double* Gb = G + (long)b * gbs;
  T* hi = reinterpret_cast<T*>(out + (long)b * obs);
  T* hiT = hi + (long)n * ld;
  const double sc = (KIND == LP_F16) ? f16_scale(*amax) : 1.0;
  auto put = [&](T* base, long idx, double x) {
    if constexpr (KIND == LP_F16) {
      const double xs = x * sc;
      const _Float16 h = (_Float16)(float)xs;
      base[idx] = h;
      base[idx + lo] = (_Float16)(float)((xs - (double)h) * 2048.0);
    } else {
      base[idx] = (T)(float)x;
    }
  };
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int r = r0 + ty + 8 * q, c = c0 + tx;
    const double x = (r < n && c < n) ? Gb[(long)r * n + c] : 0.0;
    t[ty + 8 * q][tx] = x;
    if (r < n) put(hi, (long)r * ld + c, x);          // row r of G, column c < ld
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int c = c0 + ty + 8 * q, r = r0 + tx;       // row c of G^T, column r
    if (c < n) put(hiT, (long)c * ld + r, t[tx][ty + 8 * q]);
  }
}

// Column j of panel b -> row j of the pre-converted operand (one workgroup
// per column): F16 first finds the column's largest entry for its scale.
template <int KIND>
__global__ __launch_bounds__(256) void k_convert_panel_pre(const double* X, long xbs, int n, long ld,
                                                           unsigned short* out, long obs, long lo, float* rs,
                                                           long rs_bs) {
  typedef typename LpStore<KIND>::T T;
  __shared__ float red[4];
  const int j = blockIdx.x, b = blockIdx.y;
  const double* x = X + (long)b * xbs + (long)j * n;
  T* o = reinterpret_cast<T*>(out + (long)b * obs) + (long)j * ld;
  double sc = 1.0;
  if constexpr (KIND == LP_F16) {
    float m = 0.0f;
    for (int i = threadIdx.x; i < n; i += 256) m = fmaxf(m, fabsf((float)x[i]));
    for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    m = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    sc = f16_scale(__float_as_uint(m));
    if (threadIdx.x == 0) rs[(long)b * rs_bs + j] = (float)sc;
  }
  for (int i = threadIdx.x; i < ld; i += 256) {
    const double v = (i < n) ? x[i] : 0.0;
    if constexpr (KIND == LP_F16) {
      const double xs = v * sc;
      const _Float16 h = (_Float16)(float)xs;
      o[i] = h;
      o[i + lo] = (_Float16)(float)((xs - (double)h) * 2048.0);
    } else {
      o[i] = (T)(float)v;
    }
  }
}

// Columns of a row-major R x C matrix (leading dimension lds, problem b at
// src + b * sbs) -> rows of a pre-converted operand: output row c holds
// column c (R values, zero-padded to pre_ld(R)).  32 columns per workgroup
// through an LDS tile (R <= kColsPreMaxR); split FP16 scales each output row
// by the power of two of its largest entry (rowscale[b * rs_bs + c]).
constexpr int kColsPreMaxR = 320;
template <int KIND>
__global__ __launch_bounds__(256) void k_convert_cols_pre(const double* src, long lds, long sbs, int R, int C,
                                                          long ld, unsigned short* out, long obs, long lo, float* rs,
                                                          long rs_bs) {
  typedef typename LpStore<KIND>::T T;
  __shared__ double t[kColsPreMaxR][33];
  const int b = blockIdx.y, c0 = blockIdx.x * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
  const double* S = src + (long)b * sbs;
  for (int r = ty; r < R; r += 8) t[r][tx] = (c0 + tx < C) ? S[(long)r * lds + c0 + tx] : 0.0;
  __syncthreads();
  T* O = reinterpret_cast<T*>(out + (long)b * obs);
  // each wave converts eight output rows (columns of the tile), one at a time
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  for (int q = 0; q < 8; ++q) {
    const int cc = w * 8 + q, c = c0 + cc;
    if (c >= C) break;
    double sc = 1.0;
    if constexpr (KIND == LP_F16) {
      float m = 0.0f;
      for (int r = lane; r < R; r += 64) m = fmaxf(m, fabsf((float)t[r][cc]));
      for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
      sc = f16_scale(__float_as_uint(m));
      if (lane == 0) rs[(long)b * rs_bs + c] = (float)sc;
    }
    T* o = O + (long)c * ld;
    for (int r = lane; r < ld; r += 64) {
      const double v = (r < R) ? t[r][cc] : 0.0;
      if constexpr (KIND == LP_F16) {
        const double xs = v * sc;
        const _Float16 h = (_Float16)(float)xs;
        o[r] = h;
        o[r + lo] = (_Float16)(float)((xs - (double)h) * 2048.0);
      } else {
        o[r] = (T)(float)v;
      }
    }
  }
}

__global__ void k_amax_clear(unsigned* out, int n) {
  if ((int)threadIdx.x < n) out[threadIdx.x] = 0u;
}

// out[which] = max(out[which], largest |x| over an R x Cn operand (FP32 bits;
// non-negative floats order like their bit patterns).  Problem blockIdx.y.
// Work items are pieces of 256 consecutive elements of a line along the
// unit-stride index (columns when the rows are unit-stride, else rows), one
// wave per item with four independent loads per lane; few workgroups, so
// that the final atomics do not queue up.
__global__ void k_operand_amax(const double* P, long s0, long s1, const int* t0, const int* t1, long bs,
                               const long* off, int R, int Cn, unsigned* out, int which) {
  __shared__ float red[4];
  const double* Pb = batch_base(P, off, bs, (int)blockIdx.y);
  const bool rows_fast = (t0 == nullptr && s0 == 1);
  const int inner = rows_fast ? R : Cn, outer = rows_fast ? Cn : R;
  const int pieces = (inner + 255) / 256;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  float m = 0.0f;
  const long items = (long)outer * pieces;
  for (long it = blockIdx.x * 4 + w; it < items; it += gridDim.x * 4) {
    const int o = (int)(it / pieces), q = (int)(it - (long)o * pieces);
    const long base = rows_fast ? off0(t1, s1, o) : off0(t0, s0, o);
    float v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = q * 256 + u * 64 + lane;
      v[u] = (i < inner) ? fabsf((float)Pb[base + (rows_fast ? (long)i : off0(t1, s1, i))]) : 0.0f;
    }
    m = fmaxf(m, fmaxf(fmaxf(v[0], v[1]), fmaxf(v[2], v[3])));
  }
  for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
  if (lane == 0) red[w] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    float r = red[0];
    for (int q = 1; q < (int)(blockDim.x >> 6); ++q) r = fmaxf(r, red[q]);
    atomicMax(out + which, __float_as_uint(r));
  }
}

// grid of k_operand_amax: about 256 workgroups in all (at least one per problem)
dim3 amax_grid(int R, int Cn, bool rows_fast, int batch) {
  const int outer = rows_fast ? Cn : R, inner = rows_fast ? R : Cn;
  const long items = (long)outer * ((inner + 255) / 256);
  const int per = (int)std::max<long>(1, std::min<long>((items + 3) / 4, 256 / std::max(1, batch)));
  return dim3((unsigned)per, (unsigned)batch);
}

template <int KIND, int BM, int BN, int WAVES_M, bool TBL>
void launch_lp_t(hipStream_t st, const KArgs& g, bool a_kc, bool b_kc, dim3 grid) {
  if (a_kc && b_kc)
    hipLaunchKernelGGL((gemm_lp_kernel<KIND, BM, BN, WAVES_M, true, true, TBL>), grid, dim3(256), 0, st, g);
  else if (a_kc && !b_kc)
    hipLaunchKernelGGL((gemm_lp_kernel<KIND, BM, BN, WAVES_M, true, false, TBL>), grid, dim3(256), 0, st, g);
  else if (!a_kc && b_kc)
    hipLaunchKernelGGL((gemm_lp_kernel<KIND, BM, BN, WAVES_M, false, true, TBL>), grid, dim3(256), 0, st, g);
  else
    hipLaunchKernelGGL((gemm_lp_kernel<KIND, BM, BN, WAVES_M, false, false, TBL>), grid, dim3(256), 0, st, g);
}

template <int KIND, int BM, int BN, int WAVES_M>
void launch_lp(hipStream_t st, const KArgs& g, bool a_kc, bool b_kc, dim3 grid) {
  if (needs_tables(g, 0x1fffffffL)) launch_lp_t<KIND, BM, BN, WAVES_M, true>(st, g, a_kc, b_kc, grid);
  else                 launch_lp_t<KIND, BM, BN, WAVES_M, false>(st, g, a_kc, b_kc, grid);
}

template <int BM, int BN, int WAVES_M>
void launch_typed(hipStream_t st, GemmType type, const KArgs& g, bool a_kc, bool b_kc, dim3 grid) {
  switch (type) {
    case GemmType::F64: launch_f64<BM, BN, WAVES_M>(st, g, a_kc, b_kc, grid); break;
    case GemmType::F32: launch_lp<LP_F32, BM, BN, WAVES_M>(st, g, a_kc, b_kc, grid); break;
    case GemmType::BF16: launch_lp<LP_BF16, BM, BN, WAVES_M>(st, g, a_kc, b_kc, grid); break;
    case GemmType::F16: launch_lp<LP_F16, BM, BN, WAVES_M>(st, g, a_kc, b_kc, grid); break;
  }
}

// Few outputs, long K (the closing contractions of expectation values): each
// workgroup sums a K-chunk of every output (<= 16 of them) and writes partials
// [chunk][batch][M][N]; splitk_reduce adds them in chunk order.
__global__ __launch_bounds__(256) void k_gemm_dot(KArgs g) {
  __shared__ double red[4][16];
  const int chunk = blockIdx.x, b = blockIdx.y, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const double* A = batch_base(g.A, g.oa, g.bsa, b);
  const double* B = batch_base(g.B, g.ob, g.bsb, b);
  const int k0 = chunk * g.kchunk, k1 = min(g.K, k0 + g.kchunk);
  const int mn = g.M * g.N;
  for (int o = 0; o < mn; ++o) {
    const int m = o / g.N, n = o % g.N;
    const long ao = off0(g.ta0, g.sa0, m), bo = off0(g.tb1, g.sb1, n);
    double acc = 0.0;
    for (int k = k0 + tid; k < k1; k += 256) acc += A[ao + off0(g.ta1, g.sa1, k)] * B[bo + off0(g.tb0, g.sb0, k)];
    for (int sft = 32; sft > 0; sft >>= 1) acc += __shfl_xor(acc, sft);
    if (lane == 0) red[w][o] = acc;
  }
  __syncthreads();
  if (tid < mn) {
    const double v = g.alpha * (((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid]);
    g.ws[(((long)chunk * g.batch + b) * g.M + tid / g.N) * g.N + tid % g.N] = v;
  }
}

// Choose the split of K so that a small output grid still fills the GPU.
// `tiles` counts the tiles of one problem of a batch: the split (and so the
// summation order) of a problem does not depend on how many are batched.
// Among the splits giving at least half a round of workgroups (K chunks of at
// least 256), take the one whose grid comes closest to whole rounds (256 CUs x
// the workgroups one CU holds: 1024 for the 64 x 64 kernels), the smaller
// split on near ties.
int choose_splits(long tiles, int K, long kRound = 1024) {
  const long kMin = kRound / 2;
  if (tiles >= kMin / 2) return 1;
  const int smax = (int)std::max<long>(1, std::min<long>(16, (long)K / 256));
  int best = 1;
  double best_fill = 0.0;
  for (int s = 1; s <= smax; ++s) {
    const long wg = tiles * s;
    if (wg < kMin && s < smax) continue;
    const double fill = (double)wg / (double)(((wg + kRound - 1) / kRound) * kRound);
    if (fill > best_fill + 0.03) {
      best = s;
      best_fill = fill;
    }
  }
  return best;
}

}  // namespace

void clear_words(hipStream_t st, unsigned* out, int n) {
  CTM_CHECK(n >= 0 && n <= 64, -1, "clear_words: at most 64 words");
  hipLaunchKernelGGL(k_amax_clear, dim3(1), dim3(64), 0, st, out, n);
  CTM_HIP(hipGetLastError());
}

void operand_amax(hipStream_t st, const Operand& P, int R, int C, int batch, unsigned* out) {
  hipLaunchKernelGGL(k_amax_clear, dim3(1), dim3(64), 0, st, out, 1);
  hipLaunchKernelGGL(k_operand_amax, amax_grid(R, C, P.t0 == nullptr && P.s0 == 1, batch), dim3(256), 0, st,
                     static_cast<const double*>(P.p), P.s0, P.s1, P.t0, P.t1, P.bs, P.bo, R, C, out, 0);
  CTM_HIP(hipGetLastError());
}

void gemm(hipStream_t st, GemmType type, int M, int N, int K, double alpha, const Operand& A,
          const Operand& B, double beta, const OutOperand& C, int batch, const GemmWorkspace& ws) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  // The kernels write 16 consecutive columns per row fragment; a column-major C
  // is produced as C^T = B^T A^T so that those writes are contiguous.
  if (C.t0 == nullptr && C.t1 == nullptr && C.s0 == 1 && C.s1 != 1 && (long)M * N > 16) {
    Operand At, Bt;
    At.p = B.p; At.s0 = B.s1; At.s1 = B.s0; At.t0 = B.t1; At.t1 = B.t0; At.bs = B.bs; At.bo = B.bo;
    At.amax = B.amax;
    Bt.p = A.p; Bt.s0 = A.s1; Bt.s1 = A.s0; Bt.t0 = A.t1; Bt.t1 = A.t0; Bt.bs = A.bs; Bt.bo = A.bo;
    Bt.amax = A.amax;
    OutOperand Ct = C;
    Ct.s0 = C.s1;
    Ct.s1 = C.s0;
    gemm(st, type, N, M, K, alpha, At, Bt, beta, Ct, batch, ws);
    return;
  }
  CTM_CHECK(type != GemmType::F16 || ws.amax != nullptr, -1, "gemm: split FP16 needs a scaling workspace");
  KArgs g{};
  const bool dot = (long)M * N <= 16 && K >= 8192;
  g.A = static_cast<const double*>(A.p);
  g.B = static_cast<const double*>(B.p);
  g.C = static_cast<double*>(C.p);
  g.sa0 = A.s0; g.sa1 = A.s1; g.ta0 = A.t0; g.ta1 = A.t1; g.bsa = A.bs;
  g.sb0 = B.s0; g.sb1 = B.s1; g.tb0 = B.t0; g.tb1 = B.t1; g.bsb = B.bs;
  g.sc0 = C.s0; g.sc1 = C.s1; g.tc0 = C.t0; g.tc1 = C.t1; g.bsc = C.bs;
  g.oa = A.bo;
  g.ob = B.bo;
  g.oc = C.bo;
  g.M = M; g.N = N; g.K = K; g.alpha = alpha; g.beta = beta; g.batch = batch;
  if (K <= 0) {   // C = beta * C
    g.splits = 1; g.kchunk = 1;
  }
  // k contiguous in memory -> walk k fastest when loading
  const bool a_kc = (A.t1 == nullptr && A.s1 == 1);
  const bool b_kc = (B.t0 == nullptr && B.s0 == 1);
  // tile shape: narrow N (sketch panels, bond-sized outputs) -> tall tiles
  // tiles: 64 x 64; 128 x 32 for narrow outputs; in FP64, 48-wide tiles when
  // 48 pads a dimension less than 64 does (chi = 144 is 3 x 48) and the other
  // one is long (these kernels hold two workgroups per CU)
  auto pad = [](int x, int t) { return ceil_div(x, t) * t - x; };
  int BM = 64, BN = 64;
  long round = 1024;
  if (N <= 48) {
    BM = 128; BN = 32;
  } else if (type == GemmType::F64 && pad(M, 48) < pad(M, 64) && N >= 512) {
    BM = 48; BN = 128; round = 512;
  } else if (type == GemmType::F64 && pad(N, 48) < pad(N, 64) && M >= 512) {
    BM = 128; BN = 48; round = 512;
  }
  long tiles = (long)ceil_div(M, BM) * ceil_div(N, BN);
  int splits = (K > 0) ? choose_splits(tiles, K, round) : 1;
  if (splits > 1 && (ws.p == nullptr || ws.elems < (size_t)splits * batch * M * N)) splits = 1;
  int kchunk = (K > 0) ? ((ceil_div(K, splits) + 15) / 16) * 16 : 16;
  if (dot) {   // FP64 dot products regardless of type: negligible work, K-chunks of 4096
    const int chunks = std::min(ceil_div(K, 4096), (int)std::min<size_t>(1024, ws.elems / ((size_t)batch * M * N)));
    CTM_CHECK(chunks >= 1, -1, "gemm: workspace too small for the dot-product path");
    g.kchunk = ceil_div(K, chunks);
    g.splits = ceil_div(K, g.kchunk);
    g.ws = ws.p;
    hipLaunchKernelGGL(k_gemm_dot, dim3(g.splits, batch), dim3(256), 0, st, g);
    CTM_HIP(hipGetLastError());
    long total = (long)batch * M * N;
    hipLaunchKernelGGL(splitk_reduce, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, st, g);
    CTM_HIP(hipGetLastError());
    return;
  }
  if (type != GemmType::F64) kchunk = ((kchunk + 31) / 32) * 32;   // whole 32-wide K steps
  splits = (K > 0) ? ceil_div(K, kchunk) : 1;
  g.splits = splits; g.kchunk = kchunk; g.ws = ws.p;
  if (type == GemmType::F16 && K > 0) {
    // operands without a known maximum are scanned into the workspace words
    if (!A.amax || !B.amax) hipLaunchKernelGGL(k_amax_clear, dim3(1), dim3(64), 0, st, ws.amax, 2);
    if (!A.amax)
      hipLaunchKernelGGL(k_operand_amax, amax_grid(M, K, g.ta0 == nullptr && g.sa0 == 1, batch), dim3(256), 0, st,
                         g.A, g.sa0, g.sa1, g.ta0, g.ta1, g.bsa, g.oa, M, K, ws.amax, 0);
    if (!B.amax)
      hipLaunchKernelGGL(k_operand_amax, amax_grid(K, N, g.tb0 == nullptr && g.sb0 == 1, batch), dim3(256), 0, st,
                         g.B, g.sb0, g.sb1, g.tb0, g.tb1, g.bsb, g.ob, K, N, ws.amax, 1);
    CTM_HIP(hipGetLastError());
    g.amaxA = A.amax ? A.amax : ws.amax;
    g.amaxB = B.amax ? B.amax : ws.amax + 1;
  }
  dim3 grid((unsigned)(ceil_div(M, BM) * ceil_div(N, BN)), (unsigned)splits, (unsigned)batch);
  if (BN == 32)      launch_typed<128, 32, 4>(st, type, g, a_kc, b_kc, grid);
  else if (BM == 48) launch_f64<48, 128, 1>(st, g, a_kc, b_kc, grid);
  else if (BN == 48) launch_f64<128, 48, 4>(st, g, a_kc, b_kc, grid);
  else               launch_typed<64, 64, 2>(st, type, g, a_kc, b_kc, grid);
  CTM_HIP(hipGetLastError());
  if (splits > 1) {
    long total = (long)batch * M * N;
    int blocks = (int)std::min<long>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(splitk_reduce, dim3(blocks), dim3(256), 0, st, g);
    CTM_HIP(hipGetLastError());
  }
}

void convert_square_pre(hipStream_t st, GemmType type, const double* G, long gbs, int n, int batch, void* out,
                        long obs, long lo, const unsigned* amax) {
  CTM_CHECK(type == GemmType::BF16 || (type == GemmType::F16 && amax), -1, "convert_square_pre: type");
  const long ld = pre_ld(n);
  const dim3 grid((unsigned)(ld / 32), (unsigned)(ld / 32), (unsigned)batch);
  auto* o = static_cast<unsigned short*>(out);
  if (type == GemmType::BF16)
    hipLaunchKernelGGL(k_convert_square_pre<LP_BF16>, grid, dim3(256), 0, st, G, gbs, n, ld, o, obs, lo, amax);
  else
    hipLaunchKernelGGL(k_convert_square_pre<LP_F16>, grid, dim3(256), 0, st, G, gbs, n, ld, o, obs, lo, amax);
  CTM_HIP(hipGetLastError());
}

void convert_panel_pre(hipStream_t st, GemmType type, const double* X, long xbs, int n, int k, int batch, void* out,
                       long obs, long lo, float* rowscale, long rs_bs) {
  CTM_CHECK(type == GemmType::BF16 || (type == GemmType::F16 && rowscale), -1, "convert_panel_pre: type");
  const long ld = pre_ld(n);
  const dim3 grid((unsigned)k, (unsigned)batch);
  auto* o = static_cast<unsigned short*>(out);
  if (type == GemmType::BF16)
    hipLaunchKernelGGL(k_convert_panel_pre<LP_BF16>, grid, dim3(256), 0, st, X, xbs, n, ld, o, obs, lo, rowscale,
                       rs_bs);
  else
    hipLaunchKernelGGL(k_convert_panel_pre<LP_F16>, grid, dim3(256), 0, st, X, xbs, n, ld, o, obs, lo, rowscale,
                       rs_bs);
  CTM_HIP(hipGetLastError());
}

void convert_cols_pre(hipStream_t st, GemmType type, const double* src, long lds, long sbs, int R, int C, int batch,
                      void* out, long obs, long lo, float* rowscale, long rs_bs) {
  CTM_CHECK(type == GemmType::BF16 || (type == GemmType::F16 && rowscale), -1, "convert_cols_pre: type");
  CTM_CHECK(R >= 1 && R <= kColsPreMaxR, -1, "convert_cols_pre: at most 320 rows");
  const long ld = pre_ld(R);
  const dim3 grid((unsigned)ceil_div(C, 32), (unsigned)batch);
  auto* o = static_cast<unsigned short*>(out);
  if (type == GemmType::BF16)
    hipLaunchKernelGGL(k_convert_cols_pre<LP_BF16>, grid, dim3(256), 0, st, src, lds, sbs, R, C, ld, o, obs, lo,
                       rowscale, rs_bs);
  else
    hipLaunchKernelGGL(k_convert_cols_pre<LP_F16>, grid, dim3(256), 0, st, src, lds, sbs, R, C, ld, o, obs, lo,
                       rowscale, rs_bs);
  CTM_HIP(hipGetLastError());
}

void gemm_pre(hipStream_t st, GemmType type, int M, int N, int Kp, double alpha, const PreOperand& A,
              const PreOperand& B, const OutOperand& C, int batch, const GemmWorkspace& ws) {
  if (M <= 0 || N <= 0 || batch <= 0) return;
  CTM_CHECK(type == GemmType::BF16 || type == GemmType::F16, -1, "gemm_pre: BF16 or F16 only");
  CTM_CHECK(Kp % 32 == 0 && A.ld % 8 == 0 && B.ld % 8 == 0 && A.ld >= Kp && B.ld >= Kp, -1,
            "gemm_pre: operand pitch");
  CTM_CHECK(C.t0 == nullptr && C.t1 == nullptr && C.bo == nullptr, -1, "gemm_pre: strided output only");
  const bool f16 = type == GemmType::F16;
  CTM_CHECK(!f16 || ((A.amax || A.rowscale) && (B.amax || B.rowscale)), -1, "gemm_pre: F16 scales");
  PArgs g{};
  g.A = static_cast<const unsigned short*>(A.p);
  g.B = static_cast<const unsigned short*>(B.p);
  g.C = static_cast<double*>(C.p);
  g.lda = A.ld; g.bsa = A.bs; g.loa = A.lo;
  g.ldb = B.ld; g.bsb = B.bs; g.lob = B.lo;
  g.sc0 = C.s0; g.sc1 = C.s1; g.bsc = C.bs;
  g.M = M; g.N = N; g.Kp = Kp; g.alpha = alpha; g.batch = batch;
  g.amaxA = A.amax; g.amaxB = B.amax;
  g.rsA = A.rowscale; g.rsB = B.rowscale; g.rsa_bs = A.rs_bs; g.rsb_bs = B.rs_bs;
  // 128 x 64 tiles with four waves (2 x 2); split FP16 with N > 128 takes
  // 128 x 192 tiles with eight waves (2 x 4), so that a row block of A (hi
  // and lo planes) is read once for all of N up to 192 (the sketch products
  // have N = k <= 192): 32.1 -> 30.5 ms of sketch products per D = 6,
  // chi = 144 sweep; BF16 measured 17.7 against 18.1 ms with the narrow tiles
  constexpr int BM = 128;
  const bool wide = f16 && N > 128;
  const int BN = wide ? 192 : 64;
  const long tiles = (long)ceil_div(M, BM) * ceil_div(N, BN);
  // split K until about 256 workgroups per problem (128 of the eight-wave
  // ones; no more than 8 ways, at least 8 k-tiles each), if the workspace
  // holds the partials; the choice does not depend on the batch, so a
  // problem gets the same arithmetic in any batch
  const long target = wide ? 128 : 256;
  int splits = 1;
  while (splits < 8 && tiles * splits < target && Kp / (32 * 2 * splits) >= 8) splits *= 2;
  if (splits > 1 && (ws.p == nullptr || ws.elems < (size_t)splits * batch * M * N)) splits = 1;
  const int kchunk = ceil_div(ceil_div(Kp, 32), splits) * 32;
  g.splits = ceil_div(Kp, kchunk);
  g.kchunk = kchunk;
  g.ws = ws.p;
  g.ws_cm = (C.s0 == 1 && C.s1 != 1) ? 1 : 0;
  const dim3 grid((unsigned)tiles, (unsigned)g.splits, (unsigned)batch);
  if (wide) {
    if (f16) hipLaunchKernelGGL((gemm_pre_kernel<LP_F16, BM, 192, 2, 4, 2>), grid, dim3(512), 0, st, g);
    else     hipLaunchKernelGGL((gemm_pre_kernel<LP_BF16, BM, 192, 2, 4, 3>), grid, dim3(512), 0, st, g);
  } else {
    if (f16) hipLaunchKernelGGL((gemm_pre_kernel<LP_F16, BM, 64, 2, 2, 4>), grid, dim3(256), 0, st, g);
    else     hipLaunchKernelGGL((gemm_pre_kernel<LP_BF16, BM, 64, 2, 2, 4>), grid, dim3(256), 0, st, g);
  }
  CTM_HIP(hipGetLastError());
  if (g.splits > 1) {
    KArgs r{};
    r.C = g.C;
    r.sc0 = C.s0; r.sc1 = C.s1; r.bsc = C.bs;
    r.M = M; r.N = N; r.batch = batch; r.beta = 0.0;
    r.splits = g.splits; r.ws = ws.p; r.ws_cm = g.ws_cm;
    const long total = (long)batch * M * N;
    const int blocks = (int)std::min<long>((total + 255) / 256, 4096);
    hipLaunchKernelGGL(splitk_reduce, dim3(blocks), dim3(256), 0, st, r);
    CTM_HIP(hipGetLastError());
  }
}

}  // namespace ctm
