// Tile kernels of one (exponentiation variant, output mode) family.
#include "tiles.h"

namespace rsaprng {
int launch_mont_gen(const KernelShape& s, const LaunchArgs& a, void* stream, int* occ) {
  return launch_family<kVariantMont, kModeGenerate>(s, a, stream, occ);
}
}  // namespace rsaprng
