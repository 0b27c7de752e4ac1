// Instantiates the lazy variant of the persistent single-source BFS kernel
// (bfs_kernel.hpp) for every slice width, slot count and group depth.
#include "bfs_kernel.hpp"

namespace blest {
namespace {

template <typename MT, int SLOTS, bool LDSVIS>
const void* sym_group(uint32_t group) {
  switch (group) {
    case 1: return reinterpret_cast<const void*>(&bfs_persistent<MT, SLOTS, kLazy, 1, LDSVIS>);
    case 2: return reinterpret_cast<const void*>(&bfs_persistent<MT, SLOTS, kLazy, 2, LDSVIS>);
    case 4: return reinterpret_cast<const void*>(&bfs_persistent<MT, SLOTS, kLazy, 4, LDSVIS>);
    default: return nullptr;
  }
}

template <typename MT, int SLOTS>
const void* sym_pick(uint32_t group, bool lds) {
  return lds ? sym_group<MT, SLOTS, true>(group) : sym_group<MT, SLOTS, false>(group);
}

template <typename MT>
const void* sym_slots(uint32_t slots, uint32_t group, bool lds, bool with8) {
  switch (slots) {
    case 1: return sym_pick<MT, 1>(group, lds);
    case 2: return sym_pick<MT, 2>(group, lds);
    case 4: return sym_pick<MT, 4>(group, lds);
    case 8: return with8 ? sym_pick<MT, 8>(group, lds) : nullptr;
    default: return nullptr;
  }
}

}  // namespace

const void* bfs_symbol_lazy(uint32_t sigma, uint32_t slots, uint32_t group, bool lds, bool packed) {
  // the packed layout exists for sigma = 8 with up to 4 slots
  if (packed) return sigma == 8 ? sym_slots<Packed8>(slots, group, lds, false) : nullptr;
  switch (sigma) {
    case 8: return sym_slots<uint8_t>(slots, group, lds, true);
    case 16: return sym_slots<uint16_t>(slots, group, lds, true);
    case 32: return sym_slots<uint32_t>(slots, group, lds, true);
    default: return nullptr;
  }
}

}  // namespace blest
