// The per-gate LDS addressing the host hands the kernels (PassDesc goff / aoff), checked over many
// circuit shapes for both precisions.  The kernels address amplitude i of group g of a gate as
//   sum over set bits k of g of goff[k]  +  (i & 1 ? aoff[0] : 0) + (i & 2 ? aoff[1] : 0),
// so for every gate of every pass:
// * goff[k] and aoff[] must be the layout's offsets of single tile bits (lds_at(1 << b)), with the
//   group bits of the tile's groups and the gate's two bits together covering every tile bit once:
//   then the groups' amplitudes are exactly the tile's elements, each once;
// * in a wave-local pass, group bits 6 and 7 (the wave index) sit on the same two tile bits for
//   every gate, and no gate of the pass touches them: each wave only ever reads and writes its own
//   quarter of the tile;
// * the layout itself is one-to-one on the 2^kMaxTileBits elements and leaves the dummy slot free.
// The host source is included so that its internal planner can be called directly.
#include "../../paper_2604_20384_amd/csrc/qhvp_host.cpp"

#include <cstdio>
#include <set>

static int g_fail = 0;
#define EXPECT(c, ...)                            \
  do {                                            \
    if (!(c)) {                                   \
      if (g_fail < 20) std::printf(__VA_ARGS__);  \
      ++g_fail;                                   \
    }                                             \
  } while (0)

int main() {
  for (int elem : {8, 16}) {
    std::set<int> image;
    const int dummy = elem == 8 ? 32 : qhvp::kDummyC128;
    const int tsp = elem == 8 ? qhvp::kTspC64 : qhvp::kTspC128;
    for (int t = 0; t < (1 << qhvp::kMaxTileBits); ++t) {
      const int a = lds_at(t, elem);
      EXPECT(image.insert(a).second, "elem %d: slot %d taken twice\n", elem, a);
      EXPECT(a < tsp, "elem %d: slot %d beyond the second array's offset %d\n", elem, a, tsp);
    }
    EXPECT(!image.count(dummy), "elem %d: dummy slot %d in use\n", elem, dummy);
    int bit_of[1 << 12];
    for (int& b : bit_of) b = -1;
    for (int b = 0; b < qhvp::kMaxTileBits; ++b) bit_of[lds_at(1 << b, elem)] = b;

    long gates = 0;
    for (int n = 2; n <= qhvp::kMaxQubits; ++n)
      for (int L : {1, 2, 3, 4, 5, 8, 13, 20, 40}) {
        auto passes = plan_circuit(n, L, nullptr);
        fill_tile_offsets(passes, elem);
        for (const auto& pd : passes) {
          const int mb = pd.mb;
          int wave_bits[2] = {-1, -1};
          for (int j = 0; j < pd.ng; ++j, ++gates) {
            const int lo = pd.tlo[j], hi = pd.thi[j];
            EXPECT(pd.aoff[j][0] == lds_at(1 << lo, elem) && pd.aoff[j][1] == lds_at(1 << hi, elem),
                   "n=%d L=%d: amplitude offsets\n", n, L);
            int pos[8];
            for (int k = 0; k < 8; ++k) {
              const int o = pd.goff[j][k];
              pos[k] = (o >= 0 && o < (1 << 12)) ? bit_of[o] : -1;
              EXPECT(pos[k] >= 0, "n=%d L=%d elem %d: goff %d is no single tile bit\n", n, L, elem, o);
            }
            // the tile's groups run over group bits 0 .. mb-3; with lo, hi they cover bits 0 .. mb-1
            std::set<int> cover = {lo, hi};
            for (int k = 0; k < mb - 2; ++k) cover.insert(pos[k]);
            EXPECT((int)cover.size() == mb && *cover.rbegin() == mb - 1 && *cover.begin() == 0,
                   "n=%d L=%d elem %d: group and gate bits do not cover the tile once\n", n, L, elem);
            if (pd.wave_local) {
              EXPECT(mb == qhvp::kMaxTileBits, "n=%d L=%d: wave-local pass on a partial tile\n", n, L);
              if (j == 0) { wave_bits[0] = pos[6]; wave_bits[1] = pos[7]; }
              EXPECT(pos[6] == wave_bits[0] && pos[7] == wave_bits[1],
                     "n=%d L=%d: wave bits move within a wave-local pass\n", n, L);
              for (int jj = 0; jj < pd.ng; ++jj)
                EXPECT(pd.tlo[jj] != pos[6] && pd.tlo[jj] != pos[7] && pd.thi[jj] != pos[6] && pd.thi[jj] != pos[7],
                       "n=%d L=%d: a gate touches a wave bit of a wave-local pass\n", n, L);
            }
          }
        }
      }
    std::printf("elem %d: %ld gates checked\n", elem, gates);
  }
  if (g_fail) {
    std::printf("FAILED %d checks\n", g_fail);
    return 1;
  }
  std::printf("LAYOUT OK\n");
  return 0;
}
