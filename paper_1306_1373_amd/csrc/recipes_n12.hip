// recipes_n12.hip -- fused codec kernels of the recipes with n = 12.
#include "codec_launch.hpp"

namespace dct {
namespace host {

int recipes_n12(const RecipeEntry **out) {
  static constexpr RecipeEntry k[] = {entry<12, 8, 8>(), entry<12, 12, 12>(), entry<12, 16, 12>()};
  *out = k;
  return static_cast<int>(sizeof(k) / sizeof(k[0]));
}

}  // namespace host
}  // namespace dct
