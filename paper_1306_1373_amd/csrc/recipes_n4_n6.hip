// recipes_n4_n6.hip -- fused codec kernels of the recipes with n = 4 and 6.
#include "codec_launch.hpp"

namespace dct {
namespace host {

int recipes_n4_n6(const RecipeEntry **out) {
  static constexpr RecipeEntry k[] = {entry<4, 8, 8>(), entry<4, 12, 12>(), entry<4, 16, 12>(),
                                      entry<6, 8, 8>(), entry<6, 12, 12>(), entry<6, 16, 12>()};
  *out = k;
  return static_cast<int>(sizeof(k) / sizeof(k[0]));
}

}  // namespace host
}  // namespace dct
