// q2x_dispatch.hip -- order buckets and (kind, precision) dispatch.
#include "q2x_internal.hpp"

namespace q2x {

#define Q2X_DECL(K, F) hipError_t launch_tiles_k##K##_f32_##F(int P, const TileArgs& a, int64_t n_tiles, hipStream_t s);
Q2X_DECL(0, 0)
Q2X_DECL(0, 1)
Q2X_DECL(1, 0)
Q2X_DECL(1, 1)
Q2X_DECL(2, 0)
Q2X_DECL(2, 1)
Q2X_DECL(3, 0)
Q2X_DECL(3, 1)
Q2X_DECL(4, 0)
Q2X_DECL(4, 1)
Q2X_DECL(5, 0)
Q2X_DECL(5, 1)
#undef Q2X_DECL

#define Q2X_EDECL(K, F) hipError_t launch_eval_k##K##_f32_##F(int P, const EvalArgs& a, int64_t n_tiles, hipStream_t s);
Q2X_EDECL(0, 0)
Q2X_EDECL(0, 1)
Q2X_EDECL(1, 0)
Q2X_EDECL(1, 1)
Q2X_EDECL(2, 0)
Q2X_EDECL(2, 1)
Q2X_EDECL(3, 0)
Q2X_EDECL(3, 1)
#undef Q2X_EDECL

// Compiled orders.  A request for order p runs the smallest bucket P >= p:
// degree n of the recursion depends only on degrees < n, so the first p+1
// degrees of a P-run equal a p-run exactly, and only n <= p is written.
static const int kBuckets[] = {4, 8, 12, 16, 20, 24, 28, 32};

int bucket_order(int p) {
  for (int b : kBuckets)
    if (b >= p) return b;
  return -1;
}

hipError_t launch_tiles(int kind, int prec, int P, const TileArgs& a, int64_t n_tiles, hipStream_t s) {
  const int f32 = (prec == Q2X_FP32_MIXED) ? 1 : 0;
  switch (kind * 2 + f32) {
    case 0: return launch_tiles_k0_f32_0(P, a, n_tiles, s);
    case 1: return launch_tiles_k0_f32_1(P, a, n_tiles, s);
    case 2: return launch_tiles_k1_f32_0(P, a, n_tiles, s);
    case 3: return launch_tiles_k1_f32_1(P, a, n_tiles, s);
    case 4: return launch_tiles_k2_f32_0(P, a, n_tiles, s);
    case 5: return launch_tiles_k2_f32_1(P, a, n_tiles, s);
    case 6: return launch_tiles_k3_f32_0(P, a, n_tiles, s);
    case 7: return launch_tiles_k3_f32_1(P, a, n_tiles, s);
    case 8: return launch_tiles_k4_f32_0(P, a, n_tiles, s);
    case 9: return launch_tiles_k4_f32_1(P, a, n_tiles, s);
    case 10: return launch_tiles_k5_f32_0(P, a, n_tiles, s);
    case 11: return launch_tiles_k5_f32_1(P, a, n_tiles, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_eval(int kind, int prec, int P, const EvalArgs& a, int64_t n_tiles, hipStream_t s) {
  const int f32 = (prec == Q2X_FP32_MIXED) ? 1 : 0;
  switch (kind * 2 + f32) {
    case 0: return launch_eval_k0_f32_0(P, a, n_tiles, s);
    case 1: return launch_eval_k0_f32_1(P, a, n_tiles, s);
    case 2: return launch_eval_k1_f32_0(P, a, n_tiles, s);
    case 3: return launch_eval_k1_f32_1(P, a, n_tiles, s);
    case 4: return launch_eval_k2_f32_0(P, a, n_tiles, s);
    case 5: return launch_eval_k2_f32_1(P, a, n_tiles, s);
    case 6: return launch_eval_k3_f32_0(P, a, n_tiles, s);
    case 7: return launch_eval_k3_f32_1(P, a, n_tiles, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace q2x
