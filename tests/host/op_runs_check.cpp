// Host check of the operator launch map (op_runs / op_run_of_block): for many
// mesh shapes, run lengths and dimensions every cell is covered exactly once
// and every run lies inside the mesh.
#include <cstdio>
#include <vector>
#include "fts_internal.h"
using namespace fts;
int main() {
    int bad = 0, ncase = 0;
    for (int dim = 2; dim <= 3; ++dim)
        for (int cpw : {1, 2, 3, 4, 5, 7, 10, 16})
            for (int m0 : {1, 2, 3, 5, 6, 8, 12, 16, 24, 32, 48})
                for (int m1 : {1, 2, 3, 7, 8, 9, 16, 48})
                    for (int m2 : {1, 2, 5, 8, 48}) {
                        if (dim == 2 && m2 != 1) continue;
                        int m[3] = {m0, m1, m2};
                        OpRuns o = op_runs(m, dim, cpw);
                        int64_t nc = (int64_t)m0 * m1 * (dim == 3 ? m2 : 1);
                        std::vector<int> seen(nc, 0);
                        for (int64_t b = 0; b < o.nblocks; ++b) {
                            int64_t c0; int na;
                            op_run_of_block(o, b, &c0, &na);
                            if (na < 1 || na > cpw || c0 < 0 || c0 + na > nc ) { bad++; break; }
                            for (int q = 0; q < na; ++q) seen[c0 + q]++;
                        }
                        for (auto v : seen) if (v != 1) { bad++; break; }
                        ncase++;
                    }
    printf("cases %d bad %d\n", ncase, bad);
    return bad != 0;
}
