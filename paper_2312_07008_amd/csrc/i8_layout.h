// LDS layout of the INT8 digit panels, shared by the INT8 pair kernels
// (pair_i8.hip, pair_i8_v.hip).  An LDS row holds one contraction chunk of one
// virtual: 2 NS slots of 16 bytes (digit t, half h -> logical slot 2t + h).  The
// physical slot is XOR-swizzled (NS = 4: 128-byte rows) or rotated by
// NS ((r >> 2) ^ (r >> 3)) & 1 (NS = 3, 5) so that the fragment reads of 8 or 16
// consecutive rows at one logical slot hit distinct banks.
#pragma once

namespace dfpt2 {
namespace i8l {

template <int NS>
__device__ inline int phys_slot(int r, int j) {
  if constexpr (NS == 4) {
    return j ^ ((r ^ (r >> 3)) & 7);
  } else {
    const int p = j + NS * (((r >> 2) ^ (r >> 3)) & 1);
    return p >= 2 * NS ? p - 2 * NS : p;
  }
}
template <int NS>
__device__ inline int logical_slot(int r, int p) {
  if constexpr (NS == 4) {
    return p ^ ((r ^ (r >> 3)) & 7);
  } else {
    const int j = p - NS * (((r >> 2) ^ (r >> 3)) & 1);
    return j < 0 ? j + 2 * NS : j;
  }
}

}  // namespace i8l
}  // namespace dfpt2
