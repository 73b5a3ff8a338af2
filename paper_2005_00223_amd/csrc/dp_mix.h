// Declarations of the mixed-precision (16-bit MFMA + FP32) kernels.
#pragma once
#include "dp_internal.h"

namespace dpk {

struct MixArgs {
  Dims d;
  int shape;                  // index into the supported embedding shapes
  int prec;                   // 0 = FP16, 1 = BF16
  const unsigned char *nets;  // packed per-net LDS images, net (t,u) at (t*ntypes+u)*net_bytes
  int64_t rows;
  const int32_t *atom_of_pos;
  const double4 *xw;
  const int32_t *nlist, *nreal;
  const double4 *rt, *dr;
  float *T32;                 // [natoms][M1][4]
  float *D32;                 // [rows][M1*M2]
  const float *dD32;          // [rows][M1*M2]
  double *force;              // [natoms][3]
  double *vir_part;           // [grid][9]
  double *net_deriv;          // optional [natoms][nnei][4]
};

int mix_shape_id(const Dims &d);
size_t mix_net_bytes(int shape);
size_t mix_lds_bytes(int shape, int ntypes, int pass);
void mix_pack_net(int shape, const double *const *W, const double *const *b, int prec, unsigned char *out);
int mix_grid(int64_t rows);
void launch_embed_mix(hipStream_t s, const MixArgs &a, int pass, int grid);

// fitting net: layers l < n16 use 16-bit products, the rest FP32
struct FitMixOffsets {
  int64_t wt16[MAXT][MAXF + 1];  // 16-bit W^T [out][in] (forward B operand)
  int64_t w16[MAXT][MAXF + 1];   // 16-bit W [in][out] (backward B operand)
  int64_t w32[MAXT][MAXF + 1];   // f32 W [in][out]
  int64_t b32[MAXT][MAXF + 1];   // f32 b [out]
};

struct FitMixArgs {
  Dims d;
  FitMixOffsets fo;           // byte offsets into w
  const unsigned char *w;
  int prec, n16;
  const int32_t *type_start;
  const int32_t *atom_of_pos;
  int64_t rows;
  const float *X0;            // D [rows][fw0]
  float *Y[MAXF + 1];         // Y[l] f32 [rows][fw[l]], l >= 1
  float *Tt[MAXF + 1];        // tanh outputs [rows][fw[l]]
  float *G[MAXF + 1];         // dE/dY[l]; G[0] = dE/dD
  double *eatom;
};
void launch_fit_mix(hipStream_t s, const FitMixArgs &a, int pass);

}  // namespace dpk
