// Column-matching masked product (shape 0): energy, plain product, FP32 and mixed forms.
#include "k1_kernels.hpp"

namespace emin {

template <class TA, class TI, class TO, int MODE, bool M1>
static int k1_short_go(const K1Shape& sh, const K1Args& a, int grid, hipStream_t s) {
#define EMIN_K1S(GG, SS)                                                           \
  if (sh.G == GG && sh.S == SS) {                                                  \
    if (sh.packed && SS <= 16)                                                     \
      k1_short<TA, TI, TO, GG, SS, MODE, M1, true><<<grid, kBlock, 0, s>>>(a);     \
    else                                                                           \
      k1_short<TA, TI, TO, GG, SS, MODE, M1, false><<<grid, kBlock, 0, s>>>(a);    \
    return 0;                                                                      \
  }
  EMIN_K1S(1, 1) EMIN_K1S(1, 2) EMIN_K1S(2, 2) EMIN_K1S(2, 4) EMIN_K1S(4, 4)
  EMIN_K1S(4, 8) EMIN_K1S(8, 8) EMIN_K1S(8, 16) EMIN_K1S(16, 16) EMIN_K1S(16, 32)
  EMIN_K1S(32, 32)
#undef EMIN_K1S
  return -1;
}


template <class TA, class TI, class TO, int MODE>
static int go_m(const K1Shape& sh, const K1Args& a, int grid, hipStream_t s) {
  if (a.m == 1) return k1_short_go<TA, TI, TO, MODE, true>(sh, a, grid, s);
  return k1_short_go<TA, TI, TO, MODE, false>(sh, a, grid, s);
}

// Returns -2 when (precision, mode) is not instantiated in this unit.
int launch_k1_short_b(int mode, int precision, const K1Shape& sh, const K1Args& a, int grid, hipStream_t s) {
  if (precision == 0 && mode == kModeEnergy) return go_m<double, double, double, kModeEnergy>(sh, a, grid, s);
  if (precision == 0 && mode == kModePlain) return go_m<double, double, double, kModePlain>(sh, a, grid, s);
  if (precision == 1 && mode == kModeIter) return go_m<float, float, float, kModeIter>(sh, a, grid, s);
  if (precision == 2 && mode == kModeInit) return go_m<double, double, float, kModeInit>(sh, a, grid, s);
  return -2;
}

}  // namespace emin
