// codec_launch.hpp -- host-side launch of the fused codec kernel under one recipe
// R(n, F, G), and the table of recipes the library is built with.  The recipe
// instantiations are spread over several translation units (they dominate the
// build); each one exports its part of the table.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "host.hpp"
#include "kernels.hpp"

namespace dct {
namespace host {

struct CodecArgs {
  const uint8_t *src;
  int W, H, src_stride, bw, nblocks;
  CodecQuant qa;
  uint8_t *dst;
  int dst_stride;
  int16_t *qcoef;
  unsigned long long *sse;
};

struct RecipeEntry {
  int n, F, G;
  void (*launch)(const CodecArgs &, hipStream_t);
  void (*tables)(int32_t *, int32_t *);
};

template <class RC>
void launch_codec(const CodecArgs &a, hipStream_t s) {
  const unsigned grid = static_cast<unsigned>((a.nblocks + kBlockThreads - 1) / kBlockThreads);
  if (a.qcoef)
    codec_kernel<RC, true><<<grid, kBlockThreads, 0, s>>>(a.src, a.W, a.H, a.src_stride, a.bw, a.nblocks, a.qa,
                                                          a.dst, a.dst_stride, a.qcoef, a.sse);
  else
    codec_kernel<RC, false><<<grid, kBlockThreads, 0, s>>>(a.src, a.W, a.H, a.src_stride, a.bw, a.nblocks, a.qa,
                                                           a.dst, a.dst_stride, nullptr, a.sse);
}

template <int N>
void copy_tables(int32_t *directions, int32_t *gains) {
  for (int r = 0; r < 3; ++r)
    for (int i = 0; i < N; ++i) directions[r * N + i] = kTablesN<N>.dir[r][i];
  for (int r = 0; r < 3; ++r) gains[r] = kTablesN<N>.gain[r];
  gains[3] = kTablesN<N>.sqrt2;
}

template <int N, int F, int G>
constexpr RecipeEntry entry() {
  return {N, F, G, &launch_codec<Recipe<N, F, G>>, &copy_tables<N>};
}

// The parts of the recipe table, in the order dct_recipe_list reports them
// (the default recipe first); each returns its entries and their count.
int recipes_default(const RecipeEntry **out);
int recipes_n4_n6(const RecipeEntry **out);
int recipes_n8_n10(const RecipeEntry **out);
int recipes_n12(const RecipeEntry **out);

}  // namespace host
}  // namespace dct
