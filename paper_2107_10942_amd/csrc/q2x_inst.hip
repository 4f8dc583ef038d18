// q2x_inst.hip -- instantiates the tile kernel for one (kind, precision) pair
// and every compiled order bucket.  Built once per pair with
// -DQ2X_INST_KIND=<q2x_kind> -DQ2X_INST_F32=<0|1> so the twelve large unrolled
// translation units compile in parallel (six kinds x two precisions).
#include "q2x_tile.hpp"

#ifndef Q2X_INST_KIND
#error "Q2X_INST_KIND must be defined"
#endif
#ifndef Q2X_INST_F32
#error "Q2X_INST_F32 must be defined"
#endif

#define Q2X_CAT2(a, b) a##b
#define Q2X_CAT(a, b) Q2X_CAT2(a, b)
#define Q2X_LAUNCHER Q2X_CAT(Q2X_CAT(launch_tiles_k, Q2X_INST_KIND), Q2X_CAT(_f32_, Q2X_INST_F32))

namespace q2x {

#if Q2X_INST_F32
using RealT = float;
#else
using RealT = double;
#endif

hipError_t Q2X_LAUNCHER(int P, const TileArgs& a, int64_t n_tiles, hipStream_t s) {
  const dim3 grid((unsigned)(n_tiles + a.n_split)), block(kTile);
  switch (P) {
#define Q2X_CASE(PP)                                                                         \
  case PP:                                                                                   \
    hipLaunchKernelGGL((q2x_tile_kernel<PP, Q2X_INST_KIND, RealT>), grid, block, 0, s, a, n_tiles); \
    break;
    Q2X_CASE(4)
    Q2X_CASE(8)
    Q2X_CASE(12)
    Q2X_CASE(16)
    Q2X_CASE(20)
    Q2X_CASE(24)
    Q2X_CASE(28)
    Q2X_CASE(32)
#undef Q2X_CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace q2x
