// Fused single-layer absorption of one site into an edge-corner product
// (the enlarged corner of Sec. 2.2 without forming the double-layer tensor).
//
// For every pair of environment indices (cp, cn) the Db x Db block
//   X[(cp, l, l'), (cn, u, u')]                      (Db = D^2 pairs ket, bra)
// is absorbed with the ket tensor and then the bra tensor:
//   Y[(l', u'), (r, dd, p)] = sum_{l,u}       X[(l,l'),(u,u')] Ak[l,u,r,dd,p]
//   G[(r, r'), (dd, d')]    = sum_{l',u',p}  Y[(l',u'),(r,dd,p)] Ab[l',u',r',d',p]
// and written to G[(cn, r, r'), (cp, dd, d')] (or its transpose).  Each wave
// takes one pair at a time: stage one reads its A fragments straight from X
// in HBM, keeps the result in LDS in the layout stage two reads, and stage
// two writes the block to G.  Ak and Ab (with Ab's legs reordered to
// [(l',u',p)][(r',d')]) stay in LDS for the whole workgroup.  X is read once
// and G written once: 2 chi^2 D^4 doubles of HBM traffic for
// 4 chi^2 D^6 d flops, against two table-addressed GEMMs with the
// intermediate Y (twice the size of X) going through HBM.
//
// MFMA v_mfma_f64_16x16x4f64: lane l supplies A[l%16][l/16] and B[l/16][l%16]
// of a 16x4 by 4x16 step and holds D[i][l%16] for i = l/16 + 4 r in register r.
#include "absorb.hpp"

#include <algorithm>

namespace ctm {
namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

constexpr int kWaves = 4;
// LDS leading dimensions are = 16 (mod 32) doubles, so that the two halves of
// a wave (k-slots 0,1 and 2,3 of a fragment read) fall on disjoint banks.
constexpr int kAkElems = 36 * 80;   // [(l,u)][(r,dd,p)], D = 6, d = 2
constexpr int kAbElems = 72 * 48;   // [(l',u',p)][(r',d')]
constexpr int kYElems = 72 * 48;    // per wave: [(l',u',p)][(r,dd)]

struct AbsorbArgs {
  const double* X;
  const double* Ak;
  const double* Ab;
  double* G;
  long n;
  int chi, DK, DB, d;
  int pairs_per_wave;
  int transposed;
};

__host__ __device__ __forceinline__ int padld(int x) { return x + ((16 - x % 32) + 32) % 32; }

// tile counts for the largest supported block (D = 6, d = 2): stage one
// 48 x 80 outputs over K = 36, stage two 48 x 48 over K = 72
constexpr int MT1 = 3, NT1 = 5, KS1 = 9, MT2 = 3, NT2 = 3, KS2 = 18;

__global__ __launch_bounds__(64 * kWaves) void k_absorb_fused(AbsorbArgs a) {
  __shared__ double sAk[kAkElems];
  __shared__ double sAb[kAbElems];
  __shared__ double sY[kWaves][kYElems];
  const int DK = a.DK, DB = a.DB, d = a.d;
  const int Db = DK * DB;
  const int P = DB * DB;          // stage-one rows (l', u')
  const int Q = DK * DK;          // stage-one K (l, u), stage-two rows (r, dd)
  const int R1 = Q * d;           // stage-one columns (r, dd, p)
  const int K2 = P * d;           // stage-two K (l', u', p)
  const int ldk = padld(R1), ldb = padld(P), ldy = padld(Q);
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  for (int e = tid; e < Q * R1; e += blockDim.x) sAk[(e / R1) * ldk + e % R1] = a.Ak[e];
  for (int e = tid; e < K2 * P; e += blockDim.x) {
    const int k = e / P, c = e % P;                    // k = (l', u', p), c = (r', d')
    const int lu = k / d, p = k % d;
    sAb[k * ldb + c] = a.Ab[((long)lu * P + c) * d + p];   // Ab[l'][u'][r'][d'][p]
  }
  __syncthreads();
  double* Ys = sY[w];
  const int r16 = lane & 15, kg = lane >> 4;
  const long npairs = (long)a.chi * a.chi;
  const long first = ((long)blockIdx.x * kWaves + w) * a.pairs_per_wave;
  // per-lane row / column coordinates (fixed for all pairs)
  int xoff[MT1];                  // stage-one A row (l', u') -> offset of (l', u') in the X block
  bool rok1[MT1];
#pragma unroll
  for (int mt = 0; mt < MT1; ++mt) {
    const int row = mt * 16 + r16;
    rok1[mt] = row < P;
    xoff[mt] = rok1[mt] ? (int)((row / DB) * a.n + row % DB) : 0;
  }
  for (int it = 0; it < a.pairs_per_wave; ++it) {   // same trip count in every wave
    const long pr = first + it;
    if (pr < npairs) {
      const int cp = (int)(pr / a.chi), cn = (int)(pr % a.chi);
      const double* Xb = a.X + (long)cp * Db * a.n + (long)cn * Db;
      // ---- stage one: Y = A1 Ak with A1[(l',u')][(l,u)] = X[(l,l'),(u,u')] ----
      d4 acc[MT1][NT1];
#pragma unroll
      for (int i = 0; i < MT1; ++i)
#pragma unroll
        for (int j = 0; j < NT1; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < KS1; ++ks) {
        const int k = ks * 4 + kg;                      // (l, u)
        const bool kok = k < Q;
        const long kx = kok ? (long)(k / DK) * DB * a.n + (k % DK) * DB : 0;
        double av[MT1], bv[NT1];
#pragma unroll
        for (int mt = 0; mt < MT1; ++mt) av[mt] = (rok1[mt] && kok) ? Xb[kx + xoff[mt]] : 0.0;
#pragma unroll
        for (int nt = 0; nt < NT1; ++nt) {
          const int col = nt * 16 + r16;
          bv[nt] = (kok && col < R1) ? sAk[k * ldk + col] : 0.0;
        }
#pragma unroll
        for (int mt = 0; mt < MT1; ++mt)
#pragma unroll
          for (int nt = 0; nt < NT1; ++nt)
            acc[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[mt], bv[nt], acc[mt][nt], 0, 0, 0);
      }
      // D[i][col], i = kg + 4 r  ->  Ys[(l',u',p)][(r,dd)]
#pragma unroll
      for (int nt = 0; nt < NT1; ++nt) {
        const int col = nt * 16 + r16;
        if (col < R1) {
          const int rd = col / d, p = col % d;
#pragma unroll
          for (int mt = 0; mt < MT1; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int i = mt * 16 + kg + 4 * r;
              if (i < P) Ys[(i * d + p) * ldy + rd] = acc[mt][nt][r];
            }
        }
      }
    }
    __syncthreads();
    if (pr < npairs) {
      const int cp = (int)(pr / a.chi), cn = (int)(pr % a.chi);
      // ---- stage two: G = Ys Ab' ----
      d4 acc[MT2][NT2];
#pragma unroll
      for (int i = 0; i < MT2; ++i)
#pragma unroll
        for (int j = 0; j < NT2; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < KS2; ++ks) {
        const int k = ks * 4 + kg;                      // (l', u', p)
        const bool kok = k < K2;
        double av[MT2], bv[NT2];
#pragma unroll
        for (int mt = 0; mt < MT2; ++mt) {
          const int row = mt * 16 + r16;                // (r, dd)
          av[mt] = (kok && row < Q) ? Ys[k * ldy + row] : 0.0;
        }
#pragma unroll
        for (int nt = 0; nt < NT2; ++nt) {
          const int col = nt * 16 + r16;                // (r', d')
          bv[nt] = (kok && col < P) ? sAb[k * ldb + col] : 0.0;
        }
#pragma unroll
        for (int mt = 0; mt < MT2; ++mt)
#pragma unroll
          for (int nt = 0; nt < NT2; ++nt)
            acc[mt][nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[mt], bv[nt], acc[mt][nt], 0, 0, 0);
      }
#pragma unroll
      for (int nt = 0; nt < NT2; ++nt) {
        const int col = nt * 16 + r16;
        if (col < P) {
          const int rb = col / DB, db = col % DB;
#pragma unroll
          for (int mt = 0; mt < MT2; ++mt)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const int i = mt * 16 + kg + 4 * r;       // (r, dd)
              if (i < Q) {
                const long nxt = (long)cn * Db + (i / DK) * DB + rb, prv = (long)cp * Db + (i % DK) * DB + db;
                if (a.transposed) a.G[prv * a.n + nxt] = acc[mt][nt][r];
                else a.G[nxt * a.n + prv] = acc[mt][nt][r];
              }
            }
        }
      }
    }
    __syncthreads();
  }
}

}  // namespace

bool absorb_fused_fits(int DK, int DB, int d) {
  const int P = DB * DB, Q = DK * DK;
  return DB > 1 && (long)Q * padld(Q * d) <= kAkElems && (long)P * d * padld(P) <= kAbElems &&
         (long)P * d * padld(Q) <= kYElems && P <= 16 * MT1 && Q * d <= 16 * NT1 && Q <= 4 * KS1 &&
         Q <= 16 * MT2 && P <= 16 * NT2 && P * d <= 4 * KS2;
}

void absorb_fused(hipStream_t st, const double* X, const double* Ak, const double* Ab, double* G, int chi,
                  int DK, int DB, int d, bool transposed) {
  CTM_CHECK(absorb_fused_fits(DK, DB, d), -1, "absorb_fused: block too large");
  AbsorbArgs a{};
  a.X = X; a.Ak = Ak; a.Ab = Ab; a.G = G;
  a.n = (long)chi * DK * DB;
  a.chi = chi; a.DK = DK; a.DB = DB; a.d = d;
  a.transposed = transposed ? 1 : 0;
  const long npairs = (long)chi * chi;
  // about 4 waves' worth of pairs per CU and round, at least one pair per wave
  a.pairs_per_wave = (int)std::max<long>(1, std::min<long>(8, npairs / (kWaves * 1024)));
  const long per_block = (long)kWaves * a.pairs_per_wave;
  const unsigned blocks = (unsigned)((npairs + per_block - 1) / per_block);
  hipLaunchKernelGGL(k_absorb_fused, dim3(blocks), dim3(64 * kWaves), 0, st, a);
  CTM_HIP(hipGetLastError());
}

}  // namespace ctm
