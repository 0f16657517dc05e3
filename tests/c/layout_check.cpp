// Host-side check of the state layout arithmetic of libwrls (no GPU call):
// for every predictor length, with and without the paper-mode history, and
// several image sizes, entry_offsets must map (pixel, entry) one-to-one onto
// the 4-byte words of one state copy; a pixel's entries 4g .. 4g + 3 must be
// one aligned 16-byte vector; every entry of a 64-pixel chunk must lie in
// that chunk's block; and the export order (P, beta, history) must map onto
// the state order (beta, P, history).
#include <cstdio>
#include <vector>

#include "wrls_internal.h"

static int fails = 0;
#define CHECK(cond, ...)                                      \
    do {                                                      \
        if (!(cond)) {                                        \
            if (fails < 20) std::printf(__VA_ARGS__);         \
            fails++;                                          \
        }                                                     \
    } while (0)

int main()
{
    using namespace wrls;
    const uint32_t sizes[] = {1, 63, 64, 65, 1000, 4097};
    for (int d = 1; d <= kMaxD; d++)
        for (int paper = 0; paper <= (d == 4 ? 1 : 0); paper++) {
            const int np = packed_floats(d);
            const int S = state_floats(d) + (paper ? 3 : 0);
            // export order -> state order is a bijection, beta first
            std::vector<int> seen(S, 0);
            for (int k = 0; k < S; k++) {
                const int i = state_entry_index(d, k);
                CHECK(i >= 0 && i < S, "d=%d: index %d of entry %d out of range\n", d, i, k);
                if (i >= 0 && i < S) seen[i]++;
                if (k >= np && k < np + 3 * d)
                    CHECK(i == k - np, "d=%d: beta entry %d at %d\n", d, k, i);
                if (k < np) CHECK(i == 3 * d + k, "d=%d: P entry %d at %d\n", d, k, i);
                if (k >= np + 3 * d) CHECK(i == k, "d=%d: history entry %d at %d\n", d, k, i);
            }
            for (int i = 0; i < S; i++) CHECK(seen[i] == 1, "d=%d: state index %d hit %d times\n", d, i, seen[i]);
            for (uint32_t n : sizes) {
                const uint32_t chunks = (n + 63) / 64;
                const uint32_t pitch = (chunks | 1u) * 64u;  // odd number of chunks, as the ABI
                const size_t words = (size_t)S * pitch;
                std::vector<unsigned char> used(words, 0);
                for (uint32_t j = 0; j < n; j++) {
                    for (int k = 0; k < S; k++) {
                        uint32_t voff, soff;
                        entry_offsets(S, d, k, j, voff, soff);
                        const size_t off = (size_t)voff + soff;
                        CHECK(off % 4 == 0 && off / 4 < words, "d=%d n=%u j=%u k=%d: offset %zu\n", d, n, j,
                              k, off);
                        if (off % 4 != 0 || off / 4 >= words) continue;
                        CHECK(!used[off / 4], "d=%d n=%u j=%u k=%d: word %zu used twice\n", d, n, j, k,
                              off / 4);
                        used[off / 4] = 1;
                        const size_t block = (size_t)(j / 64) * S * 256;
                        CHECK(off >= block && off < block + (size_t)S * 256,
                              "d=%d n=%u j=%u k=%d: outside its chunk\n", d, n, j, k);
                        const int i = state_entry_index(d, k);
                        if (i < 4 * vec_planes(S)) {
                            CHECK((off - (size_t)(i % 4) * 4) % 16 == 0 &&
                                      off - (size_t)(i % 4) * 4 == (size_t)vslot(j, S) + vgroup(i / 4),
                                  "d=%d n=%u j=%u k=%d: not in its 16-byte vector\n", d, n, j, k);
                        } else {
                            CHECK(off == (size_t)sslot(j, S) + sgroup(S, i - 4 * vec_planes(S)),
                                  "d=%d n=%u j=%u k=%d: scalar entry misplaced\n", d, n, j, k);
                        }
                    }
                }
            }
        }
    std::printf(fails ? "layout check: %d failures\n" : "layout check: ok\n", fails);
    return fails ? 1 : 0;
}
