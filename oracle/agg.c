/* Oracle aggregation for smoothed aggregation (CPU, serial, plain C).
 *
 * TEST INFRASTRUCTURE ONLY: called from the Python oracle through ctypes.
 *
 * The paper (Sec. 3.2) lumps strongly connected nodes into aggregates
 * ("supernodes") following Vanek's smoothed aggregation; it does not fix the
 * aggregation algorithm.  The reading used here:
 *   roots   = the lexicographically-first maximal distance-2 independent set of
 *             the strength graph S, nodes taken in increasing key
 *             kappa(i) = (h(i), i), h = MurmurHash3's 32-bit finaliser;
 *   pass 1  = every root plus its strong neighbours that are not roots
 *             (roots are >= 3 apart, so such a neighbour touches one root);
 *   pass 2  = every node still free joins the aggregate of a strong neighbour
 *             placed in pass 1, taking the neighbour whose root has the
 *             smallest key;
 *   ids     = aggregates numbered by increasing root node index.
 * Nodes without strong neighbours are their own roots (singletons).
 */
#include <stdint.h>
#include <stdlib.h>

uint32_t oracle_fmix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

static const uint32_t* g_keys;

static int cmp_key(const void* a, const void* b) {
    int32_t i = *(const int32_t*)a, j = *(const int32_t*)b;
    uint32_t ki = g_keys[i], kj = g_keys[j];
    if (ki != kj) return ki < kj ? -1 : 1;
    return (i > j) - (i < j);
}

/* S: symmetric strength graph without self loops, CSR (rowptr n+1, col).
 * Outputs: agg[n] aggregate id, is_root[n].  Returns the number of aggregates,
 * or -1 if some node is left unaggregated (cannot happen for a symmetric S). */
int64_t oracle_aggregate(int64_t n, const int64_t* rowptr, const int32_t* col,
                         int32_t* agg, uint8_t* is_root) {
    uint32_t* key = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1));
    int32_t* order = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    uint8_t* state = (uint8_t*)calloc((size_t)(n > 0 ? n : 1), 1);  /* 0 free, 1 root, 2 excluded */
    int32_t* root_of = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        key[i] = oracle_fmix32((uint32_t)i);
        order[i] = (int32_t)i;
    }
    g_keys = key;
    qsort(order, (size_t)n, sizeof(int32_t), cmp_key);

    /* greedy maximal distance-2 independent set in key order */
    for (int64_t t = 0; t < n; ++t) {
        int32_t u = order[t];
        if (state[u] != 0) continue;
        state[u] = 1;
        for (int64_t a = rowptr[u]; a < rowptr[u + 1]; ++a) {
            int32_t v = col[a];
            if (state[v] == 0) state[v] = 2;
            for (int64_t b = rowptr[v]; b < rowptr[v + 1]; ++b) {
                int32_t w = col[b];
                if (state[w] == 0) state[w] = 2;
            }
        }
    }

    /* aggregate ids by increasing root index */
    int64_t n_agg = 0;
    for (int64_t i = 0; i < n; ++i) {
        is_root[i] = state[i] == 1;
        agg[i] = -1;
        root_of[i] = -1;
        if (state[i] == 1) {
            agg[i] = (int32_t)n_agg++;
            root_of[i] = (int32_t)i;
        }
    }
    /* pass 1: neighbours of roots */
    for (int64_t i = 0; i < n; ++i) {
        if (state[i] == 1) continue;
        for (int64_t a = rowptr[i]; a < rowptr[i + 1]; ++a) {
            int32_t v = col[a];
            if (state[v] == 1) { agg[i] = agg[v]; root_of[i] = v; break; }
        }
    }
    /* pass 2: join the pass-1 neighbour whose root has the smallest key */
    int32_t* agg1 = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    int32_t* root1 = (int32_t*)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) { agg1[i] = agg[i]; root1[i] = root_of[i]; }
    int64_t missing = 0;
    for (int64_t i = 0; i < n; ++i) {
        if (agg1[i] >= 0) continue;
        int32_t best = -1;
        for (int64_t a = rowptr[i]; a < rowptr[i + 1]; ++a) {
            int32_t v = col[a];
            if (agg1[v] < 0) continue;
            int32_t r = root1[v];
            if (best < 0 || key[r] < key[best] || (key[r] == key[best] && r < best)) best = r;
        }
        if (best < 0) { ++missing; continue; }
        agg[i] = agg1[best];
        root_of[i] = best;
    }
    free(agg1); free(root1); free(key); free(order); free(state); free(root_of);
    return missing ? -1 : n_agg;
}
