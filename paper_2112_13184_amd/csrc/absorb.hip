// Fused single-layer absorption of one site into an edge-corner product
// (the enlarged corner of Sec. 2.2 without forming the double-layer tensor).
//
// For every pair of environment indices (cp, cn) the Db x Db block
//   X[(cp, l, l'), (cn, u, u')]                      (Db = D^2 pairs ket, bra)
// is absorbed with the ket tensor and then the bra tensor:
//   Y[(l', u'), (p, r, dd)] = sum_{l,u}       X[(l,l'),(u,u')] Ak[l,u,r,dd,p]
//   G[(r, dd), (r', d')]    = sum_{l',u',p}  Y[(l',u'),(p,r,dd)] Ab[l',u',r',d',p]
// and written to G[(cn, r, r'), (cp, dd, d')] (or its transpose).  X is read
// once and G written once: 2 chi^2 D^4 doubles of HBM traffic for
// 4 chi^2 D^6 d flops.
//
// MFMA v_mfma_f64_16x16x4f64: lane l supplies A[l%16][l/16] and B[l/16][l%16]
// of a 16x4 by 4x16 step and holds D[i][l%16] for i = l/16 + 4 r in register r.
// Stage one orders its columns as (p, (r, dd)) with (r, dd) padded to 48, so
// that its accumulator for row block mt, column tile nt and register r is,
// lane by lane, the A fragment of stage two for (r, dd) tile nt % 3 and the
// four k values (l', u') = 16 mt + 4 r + l/16 at p = nt / 3.  Y therefore
// never leaves registers (one p at a time, to stay within 256 registers and
// keep two waves per SIMD): each wave takes its pairs on its own, with no
// LDS traffic but the B fragments and no barrier.  Ak and Ab (legs
// reordered) stay in LDS for the whole workgroup.
#include "absorb.hpp"

#include <algorithm>

namespace ctm {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
// Tile counts: NR tiles of 16 over (r, dd), (l', u') and (r', d'), KS1 k steps
// of 4 over (l, u).  D <= 4: one tile (D^2 <= 16), four waves per SIMD.
// D = 5: D^2 = 25 padded to 32 (2 tiles), three waves per SIMD (LDS).
// D <= 6: D^2 <= 36 padded to 48 (3 tiles), two waves per SIMD.  D <= 8: 4 tiles, no padding at D = 8; the two accumulator sets take
// 256 registers, so one wave per SIMD, and Ak, Ab take 152 KB of LDS.
// LDS leading dimensions are = 16 (mod 32) doubles, so that the two halves of
// a wave (k-slots 0,1 and 2,3 of a fragment read) fall on disjoint banks.
template <int NR_, int KS1_, int ABLD_, int WPE_>
struct AbsorbShape {
  static constexpr int NR = NR_;
  static constexpr int RD = 16 * NR;            // (r, dd) padded
  static constexpr int MT1 = NR;                // stage one row tiles: (l', u') < 16 NR
  static constexpr int KS1 = KS1_;              // stage one k steps: (l, u) < 4 KS1
  static constexpr int NT2 = NR;                // stage two column tiles: (r', d') < 16 NR
  static constexpr int AKLD = 2 * RD + 16;      // [(l,u)][(p, r, dd)]
  static constexpr int ABLD = ABLD_;            // [((l',u'), p)][(r',d')]
  static constexpr int AKE = 4 * KS1 * AKLD;
  static constexpr int ABE = 16 * MT1 * 2 * ABLD;
  static constexpr int WPE = WPE_;
  static constexpr int MAXQ = 4 * KS1 < RD ? 4 * KS1 : RD;   // largest (l, u) count
  static constexpr int MAXP = 16 * NR;                       // largest (l', u') count
};
using ShapeD4 = AbsorbShape<1, 4, 48, 4>;
using ShapeD5 = AbsorbShape<2, 7, 48, 3>;
using ShapeD6 = AbsorbShape<3, 9, 48, 2>;
using ShapeD8 = AbsorbShape<4, 16, 80, 1>;

struct AbsorbArgs {
  const double* X;
  const double* Ak;
  const double* Ab;
  double* G;
  // one problem per blockIdx.y: per-problem element offsets from the bases
  // above (device arrays; null for a single problem)
  const long* xo;
  const long* ako;
  const long* abo;
  const long* go;
  // largest |G| (FP32 bits, atomic max) of each problem: amaxp[b] (device
  // table) or amax1 for a single problem; null: not computed
  unsigned* const* amaxp;
  unsigned* amax1;
  long n;
  int chi, DK, DB, d;
  int transposed;
};

// MAX: also return the largest |G| (a separate instantiation, so that the
// plain form keeps its registers for the accumulators)
template <class S, bool MAX>
__global__ __launch_bounds__(64 * kWaves) __attribute__((amdgpu_waves_per_eu(S::WPE))) void k_absorb_fused(
    AbsorbArgs a) {
  constexpr int NR = S::NR, kRD = S::RD, MT1 = S::MT1, KS1 = S::KS1, NT2 = S::NT2;
  constexpr int kAkLd = S::AKLD, kAbLd = S::ABLD, kAkElems = S::AKE, kAbElems = S::ABE;
  __shared__ double sAk[kAkElems];
  __shared__ double sAb[kAbElems];
  const int bz = blockIdx.y;
  const double* Xg = a.X + (a.xo ? a.xo[bz] : 0);
  const double* Akg = a.Ak + (a.ako ? a.ako[bz] : 0);
  const double* Abg = a.Ab + (a.abo ? a.abo[bz] : 0);
  double* Gg = a.G + (a.go ? a.go[bz] : 0);
  const int DK = a.DK, DB = a.DB, d = a.d;
  const int Db = DK * DB;
  const int P = DB * DB;          // (l', u') and (r', d')
  const int Q = DK * DK;          // (l, u) and (r, dd)
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  // zero padding everywhere outside the tensors
  for (int e = tid; e < kAkElems; e += blockDim.x) {
    const int k = e / kAkLd, c = e % kAkLd;          // c = p * 48 + (r, dd)
    const int p = c / kRD, rd = c % kRD;
    sAk[e] = (k < Q && p < d && rd < Q && c < 2 * kRD) ? Akg[((long)k * Q + rd) * d + p] : 0.0;
  }
  for (int e = tid; e < kAbElems; e += blockDim.x) {
    const int row = e / kAbLd, c = e % kAbLd;        // row = (l', u') * 2 + p, c = (r', d')
    const int lu = row >> 1, p = row & 1;
    sAb[e] = (lu < P && p < d && c < P) ? Abg[((long)lu * P + c) * d + p] : 0.0;
  }
  __syncthreads();
  const int r16 = lane & 15, kg = lane >> 4;
  // stage one A row (l', u') of this lane -> offset in the X block
  int xoff[MT1];
  bool rok[MT1];
#pragma unroll
  for (int mt = 0; mt < MT1; ++mt) {
    const int row = mt * 16 + r16;
    rok[mt] = row < P;
    xoff[mt] = rok[mt] ? (int)((row / DB) * a.n + row % DB) : 0;
  }
  const long npairs = (long)a.chi * a.chi;
  const long nwaves = (long)gridDim.x * kWaves;
  unsigned* amax = MAX ? (a.amaxp ? a.amaxp[bz] : a.amax1) : nullptr;
  double gmax = 0.0;
  for (long pr = (long)blockIdx.x * kWaves + w; pr < npairs; pr += nwaves) {
    const int cp = (int)(pr / a.chi), cn = (int)(pr % a.chi);
    const double* Xb = Xg + (long)cp * Db * a.n + (long)cn * Db;
    d4 acc2[NR][NT2];
#pragma unroll
    for (int i = 0; i < NR; ++i)
#pragma unroll
      for (int j = 0; j < NT2; ++j) acc2[i][j] = d4{0.0, 0.0, 0.0, 0.0};
    // one physical index p at a time: stage one gives Y[(l',u'), (p, r, dd)]
    // (X is read again for the second p, from L2), stage two consumes it
    for (int p = 0; p < d; ++p) {
      // ---- stage one: Y_p = A1 Ak_p with A1[(l',u')][(l,u)] = X[(l,l'),(u,u')] ----
      d4 acc1[MT1][NR];
#pragma unroll
      for (int i = 0; i < MT1; ++i)
#pragma unroll
        for (int j = 0; j < NR; ++j) acc1[i][j] = d4{0.0, 0.0, 0.0, 0.0};
      // three k steps unrolled: loads in flight for a third of the block,
      // so that the accumulators and fragments fit 256 registers
#pragma unroll 3
      for (int ks = 0; ks < KS1; ++ks) {
        const int k = ks * 4 + kg;                      // (l, u)
        const bool kok = k < Q;
        const long kx = kok ? (long)(k / DK) * DB * a.n + (k % DK) * DB : 0;
        double av[MT1], bv[NR];
#pragma unroll
        for (int mt = 0; mt < MT1; ++mt) av[mt] = (rok[mt] && kok) ? Xb[kx + xoff[mt]] : 0.0;
#pragma unroll
        for (int nt = 0; nt < NR; ++nt) bv[nt] = sAk[k * kAkLd + p * kRD + nt * 16 + r16];
#pragma unroll
        for (int mt = 0; mt < MT1; ++mt)
#pragma unroll
          for (int nt = 0; nt < NR; ++nt)
            acc1[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[mt], bv[nt], acc1[mt][nt], 0, 0, 0);
      }
      // ---- stage two: G[(r,dd)][(r',d')] += sum over (l',u') of Y_p Ab_p ----
#pragma unroll
      for (int mt = 0; mt < MT1; ++mt)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          // k slots past (l', u') = P hold zero rows of Y_p: skip them (the
          // sums are unchanged; at D = 6 this drops a quarter of stage two)
          if (mt * 16 + 4 * r >= P) continue;
          const int lu = mt * 16 + 4 * r + kg;          // (l', u') of this lane's k slot
          double bv[NT2];
#pragma unroll
          for (int nt = 0; nt < NT2; ++nt) bv[nt] = sAb[(lu * 2 + p) * kAbLd + nt * 16 + r16];
#pragma unroll
          for (int m2 = 0; m2 < NR; ++m2)
#pragma unroll
            for (int nt = 0; nt < NT2; ++nt)
              acc2[m2][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(acc1[mt][m2][r], bv[nt], acc2[m2][nt], 0, 0, 0);
        }
    }
#pragma unroll
    for (int nt = 0; nt < NT2; ++nt) {
      const int col = nt * 16 + r16;                    // (r', d')
      if (col < P) {
        const int rb = col / DB, db = col % DB;
#pragma unroll
        for (int m2 = 0; m2 < NR; ++m2)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const int i = m2 * 16 + kg + 4 * r;         // (r, dd)
            if (i < Q) {
              const long nxt = (long)cn * Db + (i / DK) * DB + rb, prv = (long)cp * Db + (i % DK) * DB + db;
              if (a.transposed) Gg[prv * a.n + nxt] = acc2[m2][nt][r];
              else Gg[nxt * a.n + prv] = acc2[m2][nt][r];
              if constexpr (MAX) gmax = fmax(gmax, fabs(acc2[m2][nt][r]));
            }
          }
      }
    }
  }
  if (MAX && amax) {
    __shared__ float red[kWaves];
    float m = (float)gmax;
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o));
    if (lane == 0) red[w] = m;
    __syncthreads();
    if (tid == 0) {
      float r = red[0];
      for (int q = 1; q < kWaves; ++q) r = fmaxf(r, red[q]);
      atomicMax(amax, __float_as_uint(r));
    }
  }
}

}  // namespace

template <class S>
static bool shape_fits(int DK, int DB, int d) {
  const int P = DB * DB, Q = DK * DK;
  return DB > 1 && d >= 1 && d <= 2 && Q <= S::MAXQ && P <= S::MAXP;
}

bool absorb_fused_fits(int DK, int DB, int d) {
  return shape_fits<ShapeD4>(DK, DB, d) || shape_fits<ShapeD5>(DK, DB, d) || shape_fits<ShapeD6>(DK, DB, d) ||
         shape_fits<ShapeD8>(DK, DB, d);
}

void absorb_fused(hipStream_t st, const double* X, const double* Ak, const double* Ab, double* G, int chi,
                  int DK, int DB, int d, bool transposed, unsigned* amax) {
  absorb_fused_batched(st, X, Ak, Ab, G, nullptr, nullptr, nullptr, nullptr, 1, chi, DK, DB, d, transposed,
                       nullptr, amax);
}

void absorb_fused_batched(hipStream_t st, const double* X, const double* Ak, const double* Ab, double* G,
                          const long* xo, const long* ako, const long* abo, const long* go, int batch, int chi,
                          int DK, int DB, int d, bool transposed, unsigned* const* amaxp, unsigned* amax1) {
  CTM_CHECK(absorb_fused_fits(DK, DB, d), -1, "absorb_fused: block too large");
  CTM_CHECK(batch >= 1 && batch <= 65535, -1, "absorb_fused: batch out of range");
  CTM_CHECK(batch == 1 || (xo && ako && abo && go), -1, "absorb_fused: a batch needs per-problem offsets");
  AbsorbArgs a{};
  a.X = X; a.Ak = Ak; a.Ab = Ab; a.G = G;
  a.xo = xo; a.ako = ako; a.abo = abo; a.go = go;
  a.amaxp = amaxp; a.amax1 = amax1;
  a.n = (long)chi * DK * DB;
  a.chi = chi; a.DK = DK; a.DB = DB; a.d = d;
  a.transposed = transposed ? 1 : 0;
  const long npairs = (long)chi * chi;
  // resident workgroups per CU on 256 CUs: four (D <= 4), three (D = 5, its
  // LDS), two (D <= 6) or one (D <= 8, its LDS); each wave strides over pairs
  const bool d4 = shape_fits<ShapeD4>(DK, DB, d);
  const bool d5 = !d4 && shape_fits<ShapeD5>(DK, DB, d);
  const bool d6 = !d4 && !d5 && shape_fits<ShapeD6>(DK, DB, d);
  const long resident = d4 ? 1024 : d5 ? 768 : d6 ? 512 : 256;
  const long per_block = kWaves;
  const unsigned blocks = (unsigned)std::min<long>(std::max<long>(1, resident / batch),
                                                   (npairs + per_block - 1) / per_block);
  const dim3 grid(blocks, batch), block(64 * kWaves);
  const bool mx = amaxp || amax1;
  if (d4 && mx)        hipLaunchKernelGGL((k_absorb_fused<ShapeD4, true>), grid, block, 0, st, a);
  else if (d4)         hipLaunchKernelGGL((k_absorb_fused<ShapeD4, false>), grid, block, 0, st, a);
  else if (d5 && mx)   hipLaunchKernelGGL((k_absorb_fused<ShapeD5, true>), grid, block, 0, st, a);
  else if (d5)         hipLaunchKernelGGL((k_absorb_fused<ShapeD5, false>), grid, block, 0, st, a);
  else if (d6 && mx)   hipLaunchKernelGGL((k_absorb_fused<ShapeD6, true>), grid, block, 0, st, a);
  else if (d6)    hipLaunchKernelGGL((k_absorb_fused<ShapeD6, false>), grid, block, 0, st, a);
  else if (mx)    hipLaunchKernelGGL((k_absorb_fused<ShapeD8, true>), grid, block, 0, st, a);
  else            hipLaunchKernelGGL((k_absorb_fused<ShapeD8, false>), grid, block, 0, st, a);
  CTM_HIP(hipGetLastError());
}

}  // namespace ctm
