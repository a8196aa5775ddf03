// recipes_n8_n10.hip -- fused codec kernels of the recipes with n = 8, and with
// n = 10 other than the default.
#include "codec_launch.hpp"

namespace dct {
namespace host {

int recipes_n8_n10(const RecipeEntry **out) {
  static constexpr RecipeEntry k[] = {entry<8, 8, 8>(), entry<8, 12, 12>(), entry<8, 16, 12>(),
                                      entry<10, 8, 8>(), entry<10, 16, 12>()};
  *out = k;
  return static_cast<int>(sizeof(k) / sizeof(k[0]));
}

}  // namespace host
}  // namespace dct
