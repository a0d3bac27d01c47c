/*
 * ORACLE (test infrastructure only; never part of the product path).
 *
 * Sequential union-find labelling of the connected components of an
 * undirected multigraph.  Definition followed: two vertices belong to the same
 * connected component iff a path joins them (Section I, first paragraph), and the
 * label of a component is its minimum vertex id (Fig. 1(b) caption and the
 * worked example in Section III-A.1).  The union-find approach (merge the
 * components joined by each edge) is the paper's own sequential baseline
 * (Section I; Rem's union-find in "Comparison with Sequential Implementation").
 *
 * Invariant used: every root is the minimum of its set.  It holds initially
 * (singletons) and is kept by always linking the larger root below the smaller
 * one, so labels[x] = find(x) is already the component minimum.
 *
 * find() uses full path compression in two passes: first walk to the root,
 * then point every vertex on the walked path directly at the root.
 */
#include <stdint.h>

static int32_t uf_find(int32_t* p, int32_t x) {
    int32_t r = x;
    while (p[r] != r) r = p[r];
    while (p[x] != r) { int32_t nx = p[x]; p[x] = r; x = nx; }
    return r;
}

/* labels[0..n) <- component minimum; returns the number of successful unions
 * (so the component count is n minus the return value), or -1 if an id lies
 * outside [0, n). */
int64_t oracle_uf_labels(const int32_t* u, const int32_t* v, int64_t m, int32_t n, int32_t* labels) {
    for (int32_t x = 0; x < n; ++x) labels[x] = x;
    int64_t unions = 0;
    for (int64_t i = 0; i < m; ++i) {
        int32_t a = u[i], b = v[i];
        if (a < 0 || a >= n || b < 0 || b >= n) return -1;
        int32_t ra = uf_find(labels, a), rb = uf_find(labels, b);
        if (ra == rb) continue;
        if (ra < rb) labels[rb] = ra; else labels[ra] = rb;
        ++unions;
    }
    for (int32_t x = 0; x < n; ++x) labels[x] = uf_find(labels, x);
    return unions;
}
