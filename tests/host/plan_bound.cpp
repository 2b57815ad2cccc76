// Host-only check of the block-step plans against the size of the split
// partials: for every block size `tot` among n particles, both precisions,
// the rows the plan writes (S x tot) must fit in blk_part_rows(n, prec).
// Prints the worst case per (prec, n) and exits non-zero on an overflow.
#include <cstdio>

#include "nbody_internal.h"

int main() {
    int bad = 0;
    for (int prec = 0; prec < 2; ++prec)
        for (int n : {1, 2, 255, 256, 257, 4096, 65536, 1 << 20}) {
            long long worst = 0, at = 0;
            for (int big_ok = 0; big_ok < 2; ++big_ok)
                for (long long tot = 1; tot <= n; ++tot) {
                    int nb, S, jc;
                    nb::blk_plan_geometry(tot, n, big_ok, prec, &nb, &S, &jc);
                    if (S < 1 || nb < 1 || (long long)jc * S < n) {
                        printf("bad geometry prec %d n %d tot %lld: nb %d S %d jc %d\n", prec, n, tot, nb, S, jc);
                        ++bad;
                    }
                    if ((long long)S * tot > worst) {
                        worst = (long long)S * tot;
                        at = tot;
                    }
                }
            const long long rows = nb::blk_part_rows(n, prec);
            printf("prec %d n %d: worst %lld rows (block of %lld), allocated %lld\n", prec, n, worst, at, rows);
            if (worst > rows) ++bad;
        }
    return bad ? 1 : 0;
}
