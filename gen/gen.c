/*
 * Seeded synthetic graph generators (test and benchmark input only).
 *
 * These produce undirected int32 edge lists (u[i], v[i]) with the shapes of the
 * paper's workload families (Section IV, Table "tab:data"): a uniform random
 * graph G(n,m), an R-MAT / Kronecker power-law graph (stands in for the Graph500
 * Kronecker graphs K1-K2 and the small-world G1-G2), a thinned 2D lattice (stands
 * in for the road network G3), and a forest-of-paths "many small components"
 * graph with bounded degree (stands in for the metagenomic de Bruijn graphs
 * M1-M4, whose degree is at most 8).  Vertex ids are randomly permuted, as the
 * paper does to remove naming bias (Section V, first paragraph).
 *
 * Nothing in this file computes connected components or any step of the
 * method: it only draws random numbers.  Every random number comes from a
 * counter-based generator (SplitMix64 finalizer applied to a keyed counter,
 * Steele, Lea & Flood, OOPSLA 2014), so each output element is a pure function
 * of (seed, stream, counter) and the result is independent of thread count.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------------- RNG */
static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
/* keyed counter hash: distinct (seed, stream) pairs give independent streams */
static inline uint64_t rng64(uint64_t seed, uint64_t stream, uint64_t ctr) {
    uint64_t key = mix64(seed * 0x9E3779B97F4A7C15ULL + mix64(stream ^ 0xD1B54A32D192ED03ULL));
    return mix64(key + ctr * 0x9E3779B97F4A7C15ULL);
}
/* uniform double in [0,1) */
static inline double rng_unit(uint64_t seed, uint64_t stream, uint64_t ctr) {
    return (double)(rng64(seed, stream, ctr) >> 11) * (1.0 / 9007199254740992.0);
}
/* uniform integer in [0, k) by multiply-high (Lemire) */
static inline uint64_t rng_below(uint64_t seed, uint64_t stream, uint64_t ctr, uint64_t k) {
    __uint128_t p = (__uint128_t)rng64(seed, stream, ctr) * (__uint128_t)k;
    return (uint64_t)(p >> 64);
}

enum { ST_PERM = 1, ST_GNM = 2, ST_RMAT = 3, ST_GRID_KEEP = 4, ST_GRID_SHUF = 5,
       ST_PL_SIZE = 6, ST_PL_TREE = 7, ST_PL_CHORD = 8, ST_BATCH = 9, ST_EDGE_SHUF = 10,
       ST_RMAT_NOISE = 11 };

/* ------------------------------------------------------------- permutation */
/* Fisher-Yates shuffle of the identity on [0,n): perm[i] = new id of vertex i. */
void gen_permutation(int64_t n, uint64_t seed, int32_t* perm) {
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    for (int64_t i = n - 1; i > 0; --i) {
        int64_t j = (int64_t)rng_below(seed, ST_PERM, (uint64_t)i, (uint64_t)(i + 1));
        int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
}

static void apply_perm(int64_t m, const int32_t* perm, int32_t* u, int32_t* v) {
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) { u[i] = perm[u[i]]; v[i] = perm[v[i]]; }
}

/* Fisher-Yates shuffle of an edge list (keeps (u[i], v[i]) pairs together). */
void gen_shuffle_edges(int64_t m, uint64_t seed, int32_t* u, int32_t* v) {
    for (int64_t i = m - 1; i > 0; --i) {
        int64_t j = (int64_t)rng_below(seed, ST_EDGE_SHUF, (uint64_t)i, (uint64_t)(i + 1));
        int32_t t = u[i]; u[i] = u[j]; u[j] = t;
        t = v[i]; v[i] = v[j]; v[j] = t;
    }
}

/* ----------------------------------------------------------------- G(n, m) */
/* m distinct unordered pairs {a,b}, a != b, drawn uniformly; the drawn
 * orientation is kept.  Rejection uses an open-addressing hash set.
 * Returns the number of edges written (m, or fewer if m > n(n-1)/2). */
int64_t gen_gnm(int32_t n, int64_t m, uint64_t seed, int32_t* u, int32_t* v) {
    if (n < 2 || m <= 0) return 0;
    int64_t maxm = (int64_t)n * (n - 1) / 2;
    if (m > maxm) m = maxm;
    uint64_t cap = 1; while (cap < (uint64_t)(2 * m + 16)) cap <<= 1;
    uint64_t* tab = (uint64_t*)malloc(cap * sizeof(uint64_t));
    if (!tab) return -1;
    memset(tab, 0xff, cap * sizeof(uint64_t));
    int64_t k = 0; uint64_t ctr = 0;
    while (k < m) {
        uint64_t r = rng64(seed, ST_GNM, ctr++);
        uint32_t a = (uint32_t)(((r & 0xffffffffULL) * (uint64_t)n) >> 32);
        uint32_t b = (uint32_t)(((r >> 32) * (uint64_t)n) >> 32);
        if (a == b) continue;
        uint64_t lo = a < b ? a : b, hi = a < b ? b : a;
        uint64_t key = (lo << 32) | hi;
        uint64_t h = mix64(key) & (cap - 1);
        int dup = 0;
        while (tab[h] != ~0ULL) { if (tab[h] == key) { dup = 1; break; } h = (h + 1) & (cap - 1); }
        if (dup) continue;
        tab[h] = key;
        u[k] = (int32_t)a; v[k] = (int32_t)b; ++k;
    }
    free(tab);
    return k;
}

/* ------------------------------------------------------------------- R-MAT */
/* Each edge picks one of four quadrants per level with probabilities
 * (a, b, c, d = 1-a-b-c), scale levels.  Duplicates and self-loops are kept.
 * Two levels share one 64-bit draw (32 bits each).  With noise > 0 each level
 * l uses perturbed probabilities (the "noisy SKG" of Seshadhri, Pinar & Kolda,
 * J. ACM 2013): mu_l ~ U[-noise, noise], a_l = a - 2 mu_l a/(a+d),
 * b_l = b + mu_l, c_l = c + mu_l, d_l = d - 2 mu_l d/(a+d).  If permute, ids
 * are then permuted by a seeded Fisher-Yates permutation. */
void gen_rmat(int scale, int64_t m, double a, double b, double c, double noise, uint64_t seed,
              int permute, int32_t* u, int32_t* v) {
    uint64_t T1[64], T2[64], T3[64];
    const double d = 1.0 - a - b - c;
    for (int l = 0; l < scale; ++l) {
        double mu = noise > 0 ? noise * (2.0 * rng_unit(seed, ST_RMAT_NOISE, (uint64_t)l) - 1.0) : 0.0;
        double al = a - 2.0 * mu * a / (a + d), bl = b + mu, cl = c + mu;
        T1[l] = (uint64_t)(al * 4294967296.0);
        T2[l] = (uint64_t)((al + bl) * 4294967296.0);
        T3[l] = (uint64_t)((al + bl + cl) * 4294967296.0);
    }
    #pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < m; ++e) {
        uint32_t x = 0, y = 0;
        uint64_t r = 0;
        for (int l = 0; l < scale; ++l) {
            uint64_t q;
            if ((l & 1) == 0) { r = rng64(seed, ST_RMAT, (uint64_t)e * 32u + (uint64_t)(l >> 1)); q = r & 0xffffffffULL; }
            else q = r >> 32;
            uint32_t bx, by;
            if (q < T1[l]) { bx = 0; by = 0; }
            else if (q < T2[l]) { bx = 0; by = 1; }
            else if (q < T3[l]) { bx = 1; by = 0; }
            else { bx = 1; by = 1; }
            x = (x << 1) | bx; y = (y << 1) | by;
        }
        u[e] = (int32_t)x; v[e] = (int32_t)y;
    }
    if (permute) {
        int64_t n = (int64_t)1 << scale;
        int32_t* perm = (int32_t*)malloc((size_t)n * sizeof(int32_t));
        gen_permutation(n, seed ^ 0x5bd1e995ULL, perm);
        apply_perm(m, perm, u, v);
        free(perm);
    }
}

/* -------------------------------------------------------- thinned 2D grid */
/* L x L lattice, vertex (r, c) has id r*L + c before permutation; each of the
 * 2L(L-1) lattice edges is kept independently with probability p.  Then ids are
 * permuted and the edge list is shuffled.  Returns the number of kept edges.
 * u, v must hold 2L(L-1) entries.  shuffle/permute flags allow the plain
 * (unpermuted) grid for closed-form tests. */
int64_t gen_grid(int32_t L, double p, uint64_t seed, int permute, int shuffle,
                 int32_t* u, int32_t* v) {
    int64_t H = (int64_t)L * (L - 1);       /* horizontal edges */
    int64_t total = 2 * H;
    uint64_t P = p >= 1.0 ? ~0ULL : (uint64_t)(p * 18446744073709551616.0);
    int maxth = 1;
#ifdef _OPENMP
    maxth = omp_get_max_threads();
#endif
    int64_t* cnt = (int64_t*)calloc((size_t)maxth + 2, sizeof(int64_t));
    int nth_used = 1;
    #pragma omp parallel num_threads(maxth)
    {
        int t = 0, nth = 1;
#ifdef _OPENMP
        t = omp_get_thread_num(); nth = omp_get_num_threads();
#endif
        int64_t chunk = (total + nth - 1) / nth;
        int64_t lo = t * chunk < total ? t * chunk : total;
        int64_t hi = lo + chunk < total ? lo + chunk : total;
        int64_t c = 0;
        for (int64_t e = lo; e < hi; ++e) if (p >= 1.0 || rng64(seed, ST_GRID_KEEP, (uint64_t)e) < P) ++c;
        cnt[t + 1] = c;
        #pragma omp barrier
        #pragma omp single
        { nth_used = nth; for (int i = 0; i < nth; ++i) cnt[i + 1] += cnt[i]; }
        int64_t w = cnt[t];
        for (int64_t e = lo; e < hi; ++e) {
            if (!(p >= 1.0 || rng64(seed, ST_GRID_KEEP, (uint64_t)e) < P)) continue;
            int64_t a, b;
            if (e < H) { int64_t r = e / (L - 1), cc = e % (L - 1); a = r * L + cc; b = a + 1; }
            else { int64_t f = e - H; int64_t r = f / L, cc = f % L; a = r * L + cc; b = a + L; }
            u[w] = (int32_t)a; v[w] = (int32_t)b; ++w;
        }
    }
    int64_t m = cnt[nth_used];
    free(cnt);
    if (permute) {
        int64_t n = (int64_t)L * L;
        int32_t* perm = (int32_t*)malloc((size_t)n * sizeof(int32_t));
        gen_permutation(n, seed ^ 0x5bd1e995ULL, perm);
        apply_perm(m, perm, u, v);
        free(perm);
    }
    if (shuffle) gen_shuffle_edges(m, seed, u, v);
    return m;
}

/* ------------------------------------------- power-law component forest */
/* Component sizes s in [1, smax] with P(s) proportional to s^-expo, drawn in
 * order until n vertices are used (the last one is truncated).  A component of
 * size s on local vertices 0..s-1 is a random path with branches: vertex i>0
 * attaches to i-1 with probability 3/4, otherwise to a uniform vertex of the
 * window [i-W, i-2]; then each vertex i >= 2 draws floor(lambda) or
 * ceil(lambda) window-local chords to [i-W, i-2].  Edges that would exceed the
 * degree cap or duplicate an existing edge are skipped. */

typedef struct { double* cdf; int32_t smax; double expo; } plsizes;

static int plsizes_init(plsizes* P, int32_t smax, double expo) {
    P->smax = smax; P->expo = expo;
    P->cdf = (double*)malloc((size_t)smax * sizeof(double));
    if (!P->cdf) return -1;
    double acc = 0.0;
    for (int32_t s = 1; s <= smax; ++s) { acc += pow((double)s, -expo); P->cdf[s - 1] = acc; }
    for (int32_t s = 0; s < smax; ++s) P->cdf[s] /= acc;
    P->cdf[smax - 1] = 1.0;
    return 0;
}
static int32_t plsizes_draw(const plsizes* P, double r) {
    int32_t lo = 0, hi = P->smax - 1;          /* first index with cdf >= r */
    while (lo < hi) { int32_t mid = (lo + hi) >> 1; if (P->cdf[mid] >= r) hi = mid; else lo = mid + 1; }
    return lo + 1;
}

/* One component: writes edges (local ids + base) if u != NULL; returns count.
 * deg and adj are caller scratch of size s and 8*s. */
static int64_t pl_component(int64_t s, int64_t base, uint64_t seed, uint64_t comp, double lambda,
                            int32_t W, int32_t maxdeg, int32_t* deg, int32_t* adj,
                            int32_t* u, int32_t* v) {
    int64_t k = 0;
    if (s < 2) return 0;
    for (int64_t i = 0; i < s; ++i) deg[i] = 0;
    uint64_t sk = seed ^ (comp * 0x9E3779B97F4A7C15ULL);
    #define PL_ADD(A, B) do { adj[(A) * 8 + deg[A]++] = (int32_t)(B); adj[(B) * 8 + deg[B]++] = (int32_t)(A); \
        if (u) { u[k] = (int32_t)(base + (A)); v[k] = (int32_t)(base + (B)); } ++k; } while (0)
    for (int64_t i = 1; i < s; ++i) {
        int64_t j = i - 1;
        uint64_t r = rng64(sk, ST_PL_TREE, (uint64_t)i);
        int64_t span = i - 1 < W - 1 ? i - 1 : W - 1;     /* window [i-1-span, i-2] */
        if ((r & 3) == 0 && span > 0) {
            int64_t jj = i - 2 - (int64_t)(((r >> 2) % (uint64_t)span));
            if (deg[jj] < maxdeg) j = jj;
        }
        PL_ADD(i, j);
    }
    int64_t nfull = (int64_t)lambda; double frac = lambda - (double)nfull;
    for (int64_t i = 2; i < s; ++i) {
        int64_t span = i - 1 < W - 1 ? i - 1 : W - 1;
        int64_t want = nfull + (rng_unit(sk, ST_PL_CHORD, (uint64_t)i * 16u) < frac ? 1 : 0);
        for (int64_t t = 0; t < want; ++t) {
            if (deg[i] >= maxdeg) break;
            int64_t j = i - 2 - (int64_t)rng_below(sk, ST_PL_CHORD, (uint64_t)i * 16u + 1u + (uint64_t)t, (uint64_t)span);
            if (deg[j] >= maxdeg) continue;
            int dup = 0;
            for (int q = 0; q < deg[i]; ++q) if (adj[i * 8 + q] == (int32_t)j) { dup = 1; break; }
            if (dup) continue;
            PL_ADD(i, j);
        }
    }
    #undef PL_ADD
    return k;
}

/* Sizes of the components: writes up to cap sizes, returns the count. */
int64_t gen_plcomp_sizes(int64_t n, double expo, int32_t smax, uint64_t seed, int32_t* sizes, int64_t cap) {
    plsizes P; if (plsizes_init(&P, smax, expo)) return -1;
    int64_t used = 0, c = 0;
    while (used < n && c < cap) {
        int64_t s = plsizes_draw(&P, rng_unit(seed, ST_PL_SIZE, (uint64_t)c));
        if (s > n - used) s = n - used;
        sizes[c++] = (int32_t)s; used += s;
    }
    free(P.cdf);
    return c;
}

/* Full forest: n vertices, returns the number of edges written (u, v must hold
 * cap entries; returns -1 if cap is too small).  If permute, ids are permuted. */
int64_t gen_plcomp(int64_t n, double expo, int32_t smax, double lambda, int32_t W, int32_t maxdeg,
                   uint64_t seed, int permute, int32_t* u, int32_t* v, int64_t cap) {
    int64_t ccap = n + 1;
    int32_t* sizes = (int32_t*)malloc((size_t)ccap * sizeof(int32_t));
    int64_t nc = gen_plcomp_sizes(n, expo, smax, seed, sizes, ccap);
    int64_t* vbase = (int64_t*)malloc((size_t)(nc + 1) * sizeof(int64_t));
    int64_t* ebase = (int64_t*)malloc((size_t)(nc + 1) * sizeof(int64_t));
    vbase[0] = 0;
    for (int64_t c = 0; c < nc; ++c) vbase[c + 1] = vbase[c] + sizes[c];
    int64_t rc = 0;
    #pragma omp parallel
    {
        int32_t* deg = (int32_t*)malloc((size_t)smax * sizeof(int32_t));
        int32_t* adj = (int32_t*)malloc((size_t)smax * 8 * sizeof(int32_t));
        #pragma omp for schedule(dynamic, 4096)
        for (int64_t c = 0; c < nc; ++c)
            ebase[c + 1] = pl_component(sizes[c], vbase[c], seed, (uint64_t)c, lambda, W, maxdeg, deg, adj, NULL, NULL);
        #pragma omp single
        {
            ebase[0] = 0;
            for (int64_t c = 0; c < nc; ++c) ebase[c + 1] += ebase[c];
            if (ebase[nc] > cap) rc = -1;
        }
        if (rc == 0) {
            #pragma omp for schedule(dynamic, 4096)
            for (int64_t c = 0; c < nc; ++c)
                pl_component(sizes[c], vbase[c], seed, (uint64_t)c, lambda, W, maxdeg, deg, adj, u + ebase[c], v + ebase[c]);
        }
        free(deg); free(adj);
    }
    int64_t m = rc == 0 ? ebase[nc] : -1;
    free(sizes); free(vbase); free(ebase);
    if (m > 0 && permute) {
        int32_t* perm = (int32_t*)malloc((size_t)n * sizeof(int32_t));
        gen_permutation(n, seed ^ 0x5bd1e995ULL, perm);
        apply_perm(m, perm, u, v);
        free(perm);
        gen_shuffle_edges(m, seed, u, v);
    }
    return m;
}

/* ------------------------------------------------------------------ batch */
/* G independent graphs.  Graph g uses seed base+g; from that seed it draws
 * log2 n ~ U[lg_lo, lg_hi], a family in {0: G(n,m), 1: R-MAT, 2: thinned grid,
 * 3: power-law components} and an average degree d ~ U[d_lo, d_hi] (G(n,m) and
 * R-MAT only; R-MAT n is rounded to a power of two, grid n = L^2).  Ids are
 * graph-local.  Two calls: gen_batch_plan fills n_g, m_g, family_g and keeps the
 * generated graphs; gen_batch_fetch copies them into the caller's concatenated
 * arrays and frees them. */
typedef struct { int32_t* u; int32_t* v; int64_t m; } bgraph;
static bgraph* g_batch = NULL;
static int32_t g_batch_G = 0;

static void batch_params(uint64_t sg, double lg_lo, double lg_hi, double d_lo, double d_hi,
                         int32_t* n, int32_t* fam, double* d, int32_t* L) {
    double x = lg_lo + (lg_hi - lg_lo) * rng_unit(sg, ST_BATCH, 0);
    *fam = (int32_t)rng_below(sg, ST_BATCH, 1, 4);
    *d = d_lo + (d_hi - d_lo) * rng_unit(sg, ST_BATCH, 2);
    *L = 0;
    if (*fam == 1) *n = 1 << (int)floor(x + 0.5);
    else if (*fam == 2) { *L = (int32_t)floor(sqrt(pow(2.0, x)) + 0.5); if (*L < 2) *L = 2; *n = (*L) * (*L); }
    else *n = (int32_t)floor(pow(2.0, x) + 0.5);
}

int gen_batch_plan(int32_t G, uint64_t seed_base, double lg_lo, double lg_hi, double d_lo, double d_hi,
                   int32_t* n_out, int64_t* m_out, int32_t* fam_out) {
    if (g_batch) return -2;
    g_batch = (bgraph*)calloc((size_t)G, sizeof(bgraph));
    g_batch_G = G;
    int err = 0;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int32_t g = 0; g < G; ++g) {
        uint64_t sg = seed_base + (uint64_t)g;
        int32_t n, fam, L; double d;
        batch_params(sg, lg_lo, lg_hi, d_lo, d_hi, &n, &fam, &d, &L);
        int64_t m = 0, cap;
        int32_t *u = NULL, *v = NULL;
        if (fam == 0) {
            cap = (int64_t)floor((double)n * d / 2.0 + 0.5);
            u = (int32_t*)malloc((size_t)(cap + 1) * 4); v = (int32_t*)malloc((size_t)(cap + 1) * 4);
            m = gen_gnm(n, cap, sg, u, v);
        } else if (fam == 1) {
            int sc = 0; while ((1 << sc) < n) ++sc;
            cap = (int64_t)floor((double)n * d / 2.0 + 0.5);
            u = (int32_t*)malloc((size_t)(cap + 1) * 4); v = (int32_t*)malloc((size_t)(cap + 1) * 4);
            gen_rmat(sc, cap, 0.57, 0.19, 0.19, 0.0, sg, 1, u, v); m = cap;
        } else if (fam == 2) {
            cap = 2 * (int64_t)L * (L - 1);
            u = (int32_t*)malloc((size_t)(cap + 1) * 4); v = (int32_t*)malloc((size_t)(cap + 1) * 4);
            m = gen_grid(L, 0.7, sg, 1, 1, u, v);
        } else {
            cap = 5 * (int64_t)n + 16;
            u = (int32_t*)malloc((size_t)(cap + 1) * 4); v = (int32_t*)malloc((size_t)(cap + 1) * 4);
            int32_t smax = n < 100000 ? n : 100000;
            m = gen_plcomp(n, 2.5, smax, 3.5, 16, 8, sg, 1, u, v, cap);
        }
        if (m < 0) err = -1;
        g_batch[g].u = u; g_batch[g].v = v; g_batch[g].m = m < 0 ? 0 : m;
        n_out[g] = n; m_out[g] = m < 0 ? 0 : m; fam_out[g] = fam;
    }
    return err;
}

int gen_batch_fetch(int32_t* u, int32_t* v) {
    if (!g_batch) return -2;
    int64_t* off = (int64_t*)malloc((size_t)(g_batch_G + 1) * sizeof(int64_t));
    off[0] = 0;
    for (int32_t g = 0; g < g_batch_G; ++g) off[g + 1] = off[g] + g_batch[g].m;
    #pragma omp parallel for schedule(dynamic, 1)
    for (int32_t g = 0; g < g_batch_G; ++g) {
        if (g_batch[g].m > 0) {
            memcpy(u + off[g], g_batch[g].u, (size_t)g_batch[g].m * 4);
            memcpy(v + off[g], g_batch[g].v, (size_t)g_batch[g].m * 4);
        }
        free(g_batch[g].u); free(g_batch[g].v);
    }
    free(off); free(g_batch); g_batch = NULL; g_batch_G = 0;
    return 0;
}

void gen_batch_discard(void) {
    if (!g_batch) return;
    for (int32_t g = 0; g < g_batch_G; ++g) { free(g_batch[g].u); free(g_batch[g].v); }
    free(g_batch); g_batch = NULL; g_batch_G = 0;
}

int gen_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
