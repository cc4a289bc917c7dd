// Node masked product through an LDS hash (shape 1), every precision and mode.
#include "k1_kernels.hpp"

namespace emin {

template <class TA, class TI, class TO, int MODE, bool M1>
static int k1_node_go(const K1Shape& sh, const K1Args& a, int grid, hipStream_t s) {
#define EMIN_K1N(BB, LL)                                                           \
  if (sh.bs == BB && sh.L == LL) {                                                 \
    k1_node<TA, TI, TO, BB, LL, MODE, M1><<<grid, kBlock, 0, s>>>(a);              \
    return 0;                                                                      \
  }
  EMIN_K1N(1, 1) EMIN_K1N(1, 2) EMIN_K1N(1, 3) EMIN_K1N(1, 4)
  EMIN_K1N(3, 1) EMIN_K1N(3, 2) EMIN_K1N(3, 3) EMIN_K1N(3, 4)
#undef EMIN_K1N
  return -1;
}


template <class TA, class TI, class TO, int MODE>
static int go_m(const K1Shape& sh, const K1Args& a, int grid, hipStream_t s) {
  if (a.m == 1) return k1_node_go<TA, TI, TO, MODE, true>(sh, a, grid, s);
  return k1_node_go<TA, TI, TO, MODE, false>(sh, a, grid, s);
}

// Returns -2 when (precision, mode) is not instantiated in this unit.
int launch_k1_hash(int mode, int precision, const K1Shape& sh, const K1Args& a, int grid, hipStream_t s) {
  if (precision == 0) {
    switch (mode) {
      case kModeIter: return go_m<double, double, double, kModeIter>(sh, a, grid, s);
      case kModeInit: return go_m<double, double, double, kModeInit>(sh, a, grid, s);
      case kModeEnergy: return go_m<double, double, double, kModeEnergy>(sh, a, grid, s);
      case kModePlain: return go_m<double, double, double, kModePlain>(sh, a, grid, s);
    }
  } else if (precision == 1) {
    if (mode == kModeIter) return go_m<float, float, float, kModeIter>(sh, a, grid, s);
  } else if (precision == 2) {
    if (mode == kModeInit) return go_m<double, double, float, kModeInit>(sh, a, grid, s);
  }
  return -2;
}

}  // namespace emin
