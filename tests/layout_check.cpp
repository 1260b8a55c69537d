// Host-only check of the FP32 fragment layout of the library (fc_internal.h):
// for every bin count N = 1..64 the (padded bin, row block) pairs enumerated
// by fp32_pair_index cover every entry of the lower triangle of an N x N
// factor exactly once (rows 4b + m - P, bins k' - P, pairs with k' < P
// skipped), never reach outside the padded tile, are numbered 0..npair-1 in
// enumeration order, and fp32_pair_kp / fp32_pair_b invert the numbering.
// Then the covariance build's gather maps: in the FP64 and FP32 records
// every entry of the lower triangle of W_q appears exactly once (the FP64
// record: in its tiles or its lead columns), in the split records twice as
// the high half and once as the low half, each at the k-sequence position of
// its row and bin; the FP64 record carries every signal bin once, and nothing
// else is gathered.
// Prints "ok" or the first failure.
#include <cstdint>
#include <cstdio>
#include <vector>

#include "fc_internal.h"

using namespace fcx;

int main()
{
    for (int N = 1; N <= 64; ++N) {
        const int ns = n_ksteps(N), P = fp32_pad(ns, N);
        if (P < 0 || P > 3) { printf("N=%d bad shift %d\n", N, P); return 1; }
        std::vector<int> hits(N * N, 0);
        int t_expect = 0, issued = 0;
        for (int kp = 0; kp < 4 * ns; ++kp) {
            for (int b = kp / 4; b < ns; ++b) {
                const int t = fp32_pair_index(ns, kp, b);
                if (t != t_expect) { printf("N=%d pair order\n", N); return 1; }
                if (fp32_pair_kp(ns, t) != kp || fp32_pair_b(ns, t) != b) {
                    printf("N=%d pair %d decodes wrongly\n", N, t);
                    return 1;
                }
                ++t_expect;
                if (kp < P) continue;  // zero columns, not issued
                ++issued;
                for (int m = 0; m < 4; ++m) {
                    const int rr = 4 * b + m - P, cc = kp - P;
                    if (rr >= 0 && rr < N && cc <= rr) hits[rr * N + cc] += 1;
                }
            }
            // blocks before the first one must not need this bin
            for (int b = 0; b < kp / 4; ++b) {
                const int last_row = 4 * b + 3 - P;
                if (kp - P <= last_row) { printf("N=%d skipped needed block\n", N); return 1; }
            }
        }
        if (t_expect != fp32_npairs(ns)) { printf("N=%d npair\n", N); return 1; }
        if (n_groups_from_ns(ns) * 64 < fp32_npairs(ns)) { printf("N=%d groups\n", N); return 1; }
        if (issued != fp32_npairs(ns) - P * ns) { printf("N=%d issued\n", N); return 1; }
        for (int r = 0; r < N; ++r)
            for (int c = 0; c < N; ++c)
                if (hits[r * N + c] != (c <= r ? 1 : 0)) {
                    printf("N=%d entry (%d,%d) covered %d times\n", N, r, c, hits[r * N + c]);
                    return 1;
                }
    }
    for (int N = 1; N <= 64; ++N) {
        const int ns = n_ksteps(N), T = N * (N + 1) / 2;
        std::vector<int16_t> m(cov_maps_size(N, ns));
        cov_maps_fill(N, ns, m.data());
        const int n64 = 2 * f64_rec_units(N), n32 = 4 * rec_w_units(ns);
        const int n16 = (int)m.size() - n64 - n32;
        const int16_t *parts[3] = {m.data(), m.data() + n64, m.data() + n64 + n32};
        const int lens[3] = {n64, n32, n16};
        for (int f = 0; f < 3; ++f) {
            std::vector<int> w(T, 0), wl(T, 0), sg(N, 0);
            for (int e = 0; e < lens[f]; ++e) {
                const int v = parts[f][e];
                if (v == kMapZero) continue;
                if (v >= 0 && v < T) ++w[v];
                else if (f == 2 && v >= kMapLo && v < kMapLo + T) ++wl[v - kMapLo];
                else if (f == 0 && v >= kMapSig && v < kMapSig + N) ++sg[v - kMapSig];
                else { printf("N=%d map %d entry %d out of range (%d)\n", N, f, e, v); return 1; }
            }
            // split records: hi twice (against d_hi and d_lo), lo once (against d_hi)
            const int want_hi = (f == 2) ? 2 : 1, want_lo = (f == 2) ? 1 : 0;
            for (int x = 0; x < T; ++x)
                if (w[x] != want_hi || wl[x] != want_lo) {
                    printf("N=%d map %d: W entry %d gathered %d + %d times\n", N, f, x, w[x], wl[x]);
                    return 1;
                }
            for (int k = 0; k < N; ++k)
                if (f == 0 && sg[k] != 1) { printf("N=%d FP64 map: signal bin %d %d times\n", N, k, sg[k]); return 1; }
        }
        // split map: the partner of every entry sits at the matching k-sequence
        // position of the B operand (bin j = p / 3, term p % 3: hi, hi, lo)
        {
            const int code = split_code(N);
            if (n16 != code_nfrag(code) * 64 * 8) { printf("N=%d split map size\n", N); return 1; }
            if (code_nb(code) != split_nb(N) || split_row0(N, split_nb(N)) != N) {
                printf("N=%d split groups\n", N);
                return 1;
            }
            int f_expect = 0;
            for (int g = 0; g < code_nb(code); ++g) {
                const int rows = split_row0(N, g + 1) - split_row0(N, g);
                if (rows < 1 || rows > 16) { printf("N=%d group %d holds %d rows\n", N, g, rows); return 1; }
                // the group's last row needs positions up to 3 row0(g+1) - 1
                if (32 * code_steps(code, g) < 3 * split_row0(N, g + 1) ||
                    32 * (code_steps(code, g) - 1) >= 3 * split_row0(N, g + 1)) {
                    printf("N=%d group %d steps\n", N, g);
                    return 1;
                }
                for (int s = 0; s < code_steps(code, g); ++s) {
                    if (code_frag(code, g, s) != f_expect++) { printf("N=%d fragment order\n", N); return 1; }
                    for (int lane = 0; lane < 64; ++lane)
                        for (int e = 0; e < 8; ++e) {
                            const int v = parts[2][(code_frag(code, g, s) * 64 + lane) * 8 + e];
                            if (v == kMapZero) continue;
                            const int p = 32 * s + 8 * (lane >> 4) + e, j = p / 3;
                            const int row = split_row0(N, g) + (lane & 15);
                            const int idx = v & (kMapLo - 1);
                            if (idx != row * (row + 1) / 2 + j || ((v & kMapLo) != 0) != (p % 3 == 2)) {
                                printf("N=%d split fragment (%d,%d) lane %d e %d\n", N, g, s, lane, e);
                                return 1;
                            }
                        }
                }
            }
            // issue order visits every fragment once
            std::vector<int> seen(code_nfrag(code), 0);
            for (int i = 0; i < code_nfrag(code); ++i) {
                const int g = code_issue_g(code, i), s = code_issue_s(code, i);
                if (g < 0 || s < 0 || s >= code_steps(code, g)) { printf("N=%d issue order\n", N); return 1; }
                ++seen[code_frag(code, g, s)];
            }
            for (int x : seen)
                if (x != 1) { printf("N=%d issue order covers a fragment %d times\n", N, x); return 1; }
        }
    }
    printf("issued pairs N=57: %d, N=38: %d, N=64: %d\n",
           fp32_npairs(n_ksteps(57)) - fp32_pad(n_ksteps(57), 57) * n_ksteps(57),
           fp32_npairs(n_ksteps(38)) - fp32_pad(n_ksteps(38), 38) * n_ksteps(38),
           fp32_npairs(n_ksteps(64)));
    printf("ok\n");
    return 0;
}
