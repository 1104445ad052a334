// Tile kernels of one (exponentiation variant, output mode) family.
#include "tiles.h"

namespace rsaprng {
int launch_crt_bat(const KernelShape& s, const LaunchArgs& a, void* stream, int* occ) {
  return launch_family<kVariantCrt, kModeBattery>(s, a, stream, occ);
}
}  // namespace rsaprng
