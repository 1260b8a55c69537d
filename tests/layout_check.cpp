// Host-only check of the FP32 fragment layout of the library (fc_internal.h):
// for every bin count N = 1..64 the (k-step, row-block) pairs enumerated by
// pair_index cover every entry of the lower triangle of an N x N factor
// exactly once, never reach outside the padded tile, and are numbered
// 0..npair-1 in enumeration order.  Prints "ok" or the first failure.
#include <cstdio>
#include <vector>

#include "fc_internal.h"

using namespace fcx;

int main()
{
    for (int N = 1; N <= 64; ++N) {
        const int ns = n_ksteps(N), nb = n_rowblocks_from_ns(ns), r0 = row_shift(ns);
        if (r0 < 0 || r0 >= 16 || r0 % 4) { printf("N=%d bad shift %d\n", N, r0); return 1; }
        std::vector<int> hits(N * N, 0);
        int t_expect = 0;
        for (int s = 0; s < ns; ++s) {
            for (int b = first_block_of_kstep(ns, s); b < nb; ++b) {
                if (pair_index(ns, s, b) != t_expect) { printf("N=%d pair order\n", N); return 1; }
                ++t_expect;
                if (s >= ksteps_of_block(ns, b)) { printf("N=%d s beyond block\n", N); return 1; }
                for (int lane = 0; lane < 64; ++lane) {
                    const int rr = 16 * b + (lane & 15) - r0, cc = 4 * s + (lane >> 4);
                    if (rr >= 0 && rr < N && cc <= rr) hits[rr * N + cc] += 1;
                }
            }
            // blocks before the first one must not need this k-step
            for (int b = 0; b < first_block_of_kstep(ns, s); ++b) {
                const int last_row = 16 * b + 15 - r0;
                if (4 * s <= last_row) { printf("N=%d skipped needed block\n", N); return 1; }
            }
        }
        if (t_expect != n_pairs_from_ns(ns)) { printf("N=%d npair\n", N); return 1; }
        for (int r = 0; r < N; ++r)
            for (int c = 0; c < N; ++c)
                if (hits[r * N + c] != (c <= r ? 1 : 0)) {
                    printf("N=%d entry (%d,%d) covered %d times\n", N, r, c, hits[r * N + c]);
                    return 1;
                }
    }
    printf("pairs N=57: %d, N=38: %d, N=64: %d\n", n_pairs_from_ns(n_ksteps(57)),
           n_pairs_from_ns(n_ksteps(38)), n_pairs_from_ns(n_ksteps(64)));
    printf("ok\n");
    return 0;
}
