// Declarations of the wide-embedding path (16-bit MFMA GEMMs over all
// neighbour pairs), used in mixed precision for embedding nets too wide for
// the register-resident kernels.
#pragma once
#include <vector>

#include "dp_mix.h"

namespace dpk {

constexpr int WIDE_MAXT = 4;                      // atom types the wide path takes
constexpr int WIDE_NETS = WIDE_MAXT * WIDE_MAXT;  // embedding nets (t, u)
constexpr int WIDE_BM = 128;                      // smallest GEMM row tile (pair rows)
constexpr int WIDE_BN = 128;                      // smallest GEMM column tile (features)
constexpr int WIDE_ROWPAD = 256;                  // rows of each net padded to the largest row tile
constexpr int WIDE_BK = 64;                       // GEMM depth per LDS stage
constexpr int WIDE_GRID = 2048;                   // workgroups of the per-atom kernels

// Per-pair activations live in row-major [rows][width] 16-bit arrays with two
// rows per real pair: row 2p holds the layer's values h(s_p), row 2p + 1 the
// tangent dh/ds at s_p.  With split storage a row holds [hi | lo], 2 width
// values (x = hi + lo, lo the 16-bit remainder), and every GEMM multiplies
// both halves by the same weights (two products, as the register-resident
// kernels do); without it one 16-bit value per feature (MIX-16 storage).  The pairs of net (t, u) occupy rows row0[t*T+u] ..,
// atom i's pairs of neighbour type u start at pair poff[i][u] of that net.
struct WideArgs {
  Dims d;
  int prec;                        // 0 = FP16, 1 = BF16
  int split;                       // 1: rows hold [hi | lo] halves
  int64_t n;                       // atoms
  const double4 *xw;               // wrapped positions, .w = type
  const int32_t *nlist, *nreal;    // formatted list, real counts [n][ntypes]
  const float4 *rt;                // environment matrix rows, FP32
  double L[3];                     // box lengths
  int32_t *poff;                   // [n][ntypes]
  int32_t *cnt;                    // [nets] pairs per net (the count pass adds)
  int64_t row0[WIDE_NETS];         // first row of each net
  const float *w0[WIDE_NETS];      // layer 0 (1 -> W1) weights and biases, FP32
  const float *b0[WIDE_NETS];
  uint16_t *X0;                    // [rows][W1 (x2 split)] layer-0 output
  const uint16_t *G;               // [rows][M1 (x2 split)] last layer output
  float *T32;                      // [n][M1][4] T / Nc
  const float *dT32;               // [n][M1][4] dE/dT of the unscaled sum
  double *force;                   // [n][3]
  double *vir_part;                // [WIDE_GRID][9]
  double *net_deriv;               // optional [n][nnei][4]
};

struct WideGemm {
  const uint16_t *A;   // [rows][K] layer input (value and tangent rows; split: [hi | lo], K = 2 Kb)
  const uint16_t *Bt;  // [N][Kb] weights, transposed (both halves of a split input use them)
  const float *bias;   // [N]
  uint16_t *Y;         // [rows][N (x2 split)] layer output
  int64_t rows;        // multiple of WIDE_ROWPAD
  int K, Kb, N;        // K, Kb % WIDE_BK == 0, N % WIDE_BN == 0
  int skip;            // 0 none, 1 identity (N == Kb), 2 doubling (N == 2 Kb)
  int split;           // 1: input and output rows hold [hi | lo]
};

// per-net byte offsets of the packed weights: layer 0 w, b (FP32); layer
// l >= 1 transposed W (16-bit, [out][in]) and b (FP32)
struct WideNet {
  int64_t w[MAXL], b[MAXL];
};

bool wide_supported(const Dims &d, const char **why);
// packs net (t, u) weights W[l] ([in][out] FP64), b[l] into buf, offsets into o
void wide_pack_net(const Dims &d, const double *const *W, const double *const *b, int prec,
                   std::vector<unsigned char> &buf, WideNet &o);
void launch_wide_count(hipStream_t s, const WideArgs &a);
void launch_wide_l0(hipStream_t s, const WideArgs &a);
void launch_wide_gemm(hipStream_t s, const WideGemm &g, int prec);
void launch_wide_T(hipStream_t s, const WideArgs &a);
void launch_wide_bwd(hipStream_t s, const WideArgs &a);

}  // namespace dpk
