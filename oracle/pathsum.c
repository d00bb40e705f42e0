/*
 * Brute-force Feynman path sum for noise-free QAOA p=1 MaxCut (oracle).
 *
 * TEST INFRASTRUCTURE ONLY: linked by the oracle's Python wrapper, never by
 * the product library.
 *
 * Each satisfying assignment of the circuit's CNF is one Feynman path and the
 * weighted count of those paths is the amplitude (Sec. 3.2.1).  For the QAOA
 * p=1 circuit (H on every qubit; per edge CNOT, RZ(2g) on the target, CNOT;
 * RX(2b) on every qubit) the paths are labelled by the bit string z after the
 * Hadamard layer, and the path weight is
 *
 *   2^{-n/2} * exp(-i g (|E| - 2 cut(z))) * cos(b)^{n-m} * (-i sin b)^m,
 *
 * where cut(z) is the number of edges with differing end bits and m = |z ^ x|
 * is the Hamming distance to the output x.  The weight depends on z only
 * through (cut, m), so this file counts the paths per (cut, m) exactly, in
 * integers, by visiting every z in Gray-code order; the Python side turns the
 * counts into the amplitude for any angles.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static int popcount64(uint64_t v) { return __builtin_popcountll(v); }

/* hist[c * (n + 1) + m] += number of z with cut(z) = c and |z ^ x| = m. */
int qkc_oracle_pathsum_hist(int n, int n_edges, const int *edges, uint64_t x,
                            uint64_t *hist) {
    if (n < 1 || n > 62 || n_edges < 0) return 1;
    int *deg = (int *)calloc((size_t)n, sizeof(int));
    int *adj = (int *)malloc(sizeof(int) * (size_t)(2 * n_edges + 1));
    int *start = (int *)calloc((size_t)n + 1, sizeof(int));
    if (!deg || !adj || !start) return 2;
    for (int e = 0; e < n_edges; ++e) {
        int a = edges[2 * e], b = edges[2 * e + 1];
        if (a < 0 || b < 0 || a >= n || b >= n || a == b) return 3;
        deg[a]++, deg[b]++;
    }
    for (int v = 0; v < n; ++v) start[v + 1] = start[v] + deg[v];
    int *fill = (int *)calloc((size_t)n, sizeof(int));
    for (int e = 0; e < n_edges; ++e) {
        int a = edges[2 * e], b = edges[2 * e + 1];
        adj[start[a] + fill[a]++] = b;
        adj[start[b] + fill[b]++] = a;
    }
    free(fill);

    const int split = n > 14 ? 10 : 0;
    const int low = n - split;
    const size_t hsz = (size_t)(n_edges + 1) * (size_t)(n + 1);
    memset(hist, 0, hsz * sizeof(uint64_t));

#pragma omp parallel
    {
        uint64_t *loc = (uint64_t *)calloc(hsz, sizeof(uint64_t));
#pragma omp for schedule(dynamic, 1)
        for (long h = 0; h < (1L << split); ++h) {
            uint64_t z = (uint64_t)h << low;
            int cut = 0;
            for (int e = 0; e < n_edges; ++e)
                cut += (int)(((z >> edges[2 * e]) ^ (z >> edges[2 * e + 1])) & 1u);
            int m = popcount64(z ^ x);
            loc[(size_t)cut * (n + 1) + m]++;
            for (uint64_t i = 1; i < (1ULL << low); ++i) {
                int b = __builtin_ctzll(i);
                int zb = (int)((z >> b) & 1u);
                for (int t = start[b]; t < start[b + 1]; ++t) {
                    int zu = (int)((z >> adj[t]) & 1u);
                    cut += (zu == zb) ? 1 : -1;
                }
                m += (((x >> b) & 1u) == (uint64_t)zb) ? 1 : -1;
                z ^= (1ULL << b);
                loc[(size_t)cut * (n + 1) + m]++;
            }
        }
#pragma omp critical
        for (size_t i = 0; i < hsz; ++i) hist[i] += loc[i];
        free(loc);
    }
    free(deg);
    free(adj);
    free(start);
    return 0;
}
