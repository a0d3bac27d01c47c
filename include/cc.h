/*
 * cc.h -- exact connected-component labelling of undirected int32 edge lists on
 * AMD Instinct MI355X (gfx950).  C ABI of libccmi.so.
 *
 * Problem (Section III-A.1, Notations): given an undirected graph G = (V, E)
 * with n = |V| vertices and m = |E| edges, label every vertex with its
 * connected component; two vertices share a component iff a path joins them
 * (Section I).  The label written for a vertex is the smallest vertex id of its
 * component (the canonical partition id of Fig. 1(b)), so the output is unique
 * and independent of the route, the thread schedule and the edge order.
 *
 * Method: the hybrid of Algorithm 2 (Section III-B).  An optional BFS from one
 * seed labels the dominant component and removes its edges; the
 * Shiloach-Vishkin style iteration of Section III-A (hook each partition to its
 * minimum neighbour, pointer-jump, drop finished work) labels the rest.  The
 * BFS step runs only when the degree distribution is classed as scale-free
 * (power-law fit, K-S statistic below tau = 0.05, Section V) or when a learned
 * router picks it.
 *
 * Conventions shared by every entry point:
 *  - Pointers named as device pointers must be device memory of the current
 *    HIP device (e.g. torch tensor storage).  Host pointers are marked "host".
 *  - The caller owns every array it passes; inputs are never modified; outputs
 *    are written only on success (on CC_ERANGE the labels are undefined).
 *  - `stream` is a hipStream_t (NULL = the legacy default stream).  All device
 *    work on the caller's arrays is enqueued on it.  Calls return after their
 *    results are complete (they read small device counters to drive their
 *    loops), i.e. they are host-synchronous with respect to `stream`.  One
 *    exception to the single stream: when the heuristic route fits the degree
 *    distribution while a first SV launch runs (lists of 2^22 edges or more,
 *    cached or caller scratch), the fit's kernel runs on a second stream the
 *    library keeps per device; it reads only the library's own scratch and
 *    has finished before the call goes on.
 *  - Scratch memory of cc_label / cc_label_ex comes from one of three
 *    places (cc_options.scratch, cc_options.workspace):
 *      the caller's device block of at least cc_workspace_size() bytes
 *        (nothing is allocated on the device; calls with their own blocks
 *        run at once from any threads and streams);
 *      stream-ordered allocations on `stream` from a memory pool the library
 *        keeps per device, freed stream-ordered before the call returns
 *        (no lock; calls on different streams run at once);
 *      by default, the library's cached per-device workspace, grown with
 *        hipMalloc and kept until cc_release_workspace(): the fastest for
 *        repeated calls, but calls that use it serialise on a per-device lock.
 *    The batched calls and the step entry points use the cached workspace.
 *    Small readbacks use pinned host buffers that the library keeps (one per
 *    call in flight).  cc_release_workspace() trims the current device's pool
 *    and frees its cached workspace; cc_shutdown() frees everything the
 *    library holds.
 *  - Return value: CC_OK (0) or a negative CC_E* code; cc_last_error() then
 *    returns a message (thread-local).  Nothing is thrown across the ABI.
 */
#ifndef CCMI_CC_H
#define CCMI_CC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CC_VERSION 10200 /* 1.2.0 */

/* ------------------------------------------------------------ status codes */
#define CC_OK 0
#define CC_EINVAL (-1)     /* bad argument: negative size, NULL with non-zero size, bad offsets/options */
#define CC_ERANGE (-2)     /* an edge endpoint lies outside [0, n) (detected on the device) */
#define CC_ENOMEM (-3)     /* device or pinned-host allocation failed */
#define CC_EHIP (-4)       /* a HIP runtime call failed; message has hipGetErrorString */
#define CC_EINTERNAL (-5)  /* pass cap reached (cc_options.max_passes) or an internal invariant failed */
#define CC_ENOROUTER (-6)  /* CC_ROUTE_ROUTER requested but no router weights are loaded */

/* ------------------------------------------------------------------ routes */
#define CC_ROUTE_AUTO 0       /* router if weights are loaded, else the degree heuristic */
#define CC_ROUTE_HEURISTIC 1  /* Algorithm 2: K-S statistic < tau -> BFS + SV, else SV */
#define CC_ROUTE_ROUTER 2     /* argmax of the MLP router's three logits */
#define CC_ROUTE_SV 3         /* force R1: plain SV, one hook attempt per edge per pass */
#define CC_ROUTE_BFS_SV 4     /* force R0: BFS from the max-degree vertex, then SV on the rest */
#define CC_ROUTE_SV_THETA 5   /* force R2: SV with up to theta hook attempts per edge per pass */

/* Whatever the route requested, the BFS step (R0) is taken only where it
 * applies: n <= 2^29 and m < 2^31 (the bucketed degree pass), and a BFS that
 * is still running after 256 levels (a component of long diameter, which
 * Section III-B does not intend it for) is abandoned before it writes any
 * label.  SV then labels the whole graph and cc_stats.route reports R1. */

/* route ids reported in cc_stats.route and used as router classes */
#define CC_R0_BFS_SV 0
#define CC_R1_SV 1
#define CC_R2_SV_THETA 2

/* scratch modes (cc_options.scratch), used when no workspace is given */
#define CC_SCRATCH_CACHED 0 /* the library's per-device workspace, kept between calls; calls serialise on it */
#define CC_SCRATCH_POOL 1   /* stream-ordered allocations on `stream` from the library's per-device pool */

typedef struct cc_options {
    int32_t route;       /* CC_ROUTE_* */
    int32_t max_passes;  /* 0: no cap (unless CCMI_MAX_PASSES=k is set in the environment, for failure
                            tests); else CC_EINTERNAL once this many SV passes ran without converging */
    double tau;          /* K-S threshold; <= 0 selects 0.05 (Section V, Table "tab:ks_stat") */
    double theta;        /* R2: hook attempts per edge per pass (an edge whose hook finds the root already
                            linked follows the link and retries); < 1 selects 8 */
    int32_t profile;     /* 1: time every kernel launch with HIP events (cc_stats.kernel_*) */
    int32_t scratch;     /* CC_SCRATCH_*; ignored when workspace is set */
    void* workspace;     /* device memory owned by the caller, used as the call's only device scratch;
                            NULL: see scratch.  Must not be used by anything else during the call. */
    int64_t workspace_bytes; /* its size: at least cc_workspace_size(m, n, route), else CC_EINVAL */
    int32_t check;       /* 1: debug checks on the device (the environment variable CCMI_CHECK=1 turns
                            them on for every call): after every SV pass, each parent link must point
                            into [0, x]; on return, the ends of every edge must carry one label and
                            labels[x] <= x, labels[labels[x]] == labels[x]; a violation fails the call
                            with CC_EINTERNAL.  More SV passes than 8 ceil(log2(n + 1)) + 64 (Section
                            III-A bounds the iterations by O(log n)) set bit 1 of cc_stats.check_flags.
                            Costs one extra read of parent[] per pass and one of the result. */
    int32_t reserved[3]; /* must be zero */
} cc_options;

/* kernel classes for cc_stats.kernel_* */
#define CC_K_SV_PASS 0     /* hook + compaction pass over active edges */
#define CC_K_SV_SHORTCUT 1 /* pointer jumping of hooked roots */
#define CC_K_SV_FINALIZE 2 /* init + final label pass */
#define CC_K_DEGREE 3      /* degree (endpoint counting) */
#define CC_K_HIST 4        /* degree histograms */
#define CC_K_CSR 5         /* CSR scan + fill */
#define CC_K_BFS 6         /* BFS levels */
#define CC_K_FILTER 7      /* BFS label + edge filter */
#define CC_K_CLASSES 8

typedef struct cc_stats {
    int32_t route;                /* route taken: CC_R0_BFS_SV, CC_R1_SV or CC_R2_SV_THETA */
    int32_t sv_passes;            /* SV passes over active edges */
    int32_t bfs_levels;           /* BFS levels expanded (R0) */
    int32_t bfs_bottom_up_levels; /* of which bottom-up */
    int32_t bfs_seed;             /* BFS seed (max degree, smallest id on ties), -1 if none */
    int32_t bfs_label;            /* minimum id of the BFS component, -1 if none */
    int64_t bfs_visited;          /* vertices reached by the BFS */
    int64_t bfs_edges_examined;   /* adjacency entries read by the BFS */
    int64_t edges_after_filter;   /* edges left for SV after the BFS step */
    int64_t max_degree;           /* when the degree pass ran, else -1 */
    double ks_statistic;          /* K-S statistic when computed, else NaN */
    double ks_alpha;              /* fitted power-law exponent, else NaN */
    int64_t ks_dmin;              /* fitted lower cutoff, else 0 */
    float router_logits[3];       /* when the router ran, else 0 */
    int32_t sv_deep_rounds;       /* flatten rounds forced by chains deeper than the
                                     64-link walk bound (0 on shallow forests) */
    int64_t active_edges[64];     /* active edges entering SV pass i (first 64 passes) */
    int64_t hooks_total;          /* successful hooks over all passes */
    double ms_predict;            /* degree pass + histograms + decision */
    double ms_csr;                /* CSR build (R0) */
    double ms_bfs;                /* BFS levels (R0) */
    double ms_filter;             /* BFS label + edge filter (R0) */
    double ms_sv;                 /* SV passes, shortcuts and finalize */
    double ms_total;              /* whole call, device time between first and last event */
    double algorithmic_bytes;     /* bytes the method must move (cost model) */
    double kernel_ms[8];          /* device time per kernel class, summed (profile = 1 only) */
    int32_t kernel_launches[8];   /* launches per kernel class (profile = 1 only) */
    double kernel_bytes[8];       /* algorithmic bytes per kernel class (profile = 1 only) */
    int64_t sv_atomics;           /* atomicMin operations issued by the SV passes */
    int64_t sv_chase_reads;       /* parent[] reads of the SV passes beyond two per active edge */
    int64_t giant_dropped;        /* edges of the first pass dropped on the bitmap of the largest tree */
    int32_t check_flags;          /* bit 0: the debug checks ran and passed; bit 1: more SV passes than
                                     check_pass_limit */
    int32_t check_pass_limit;     /* 8 ceil(log2(n + 1)) + 64 when the checks ran, else 0 */
    int32_t sv_hubs;              /* vertices of highest degree whose largest-tree probes the first pass
                                     answered from LDS (degrees known and a chunked first pass), else 0 */
} cc_stats;

/* Fills *opt with the defaults (route AUTO, no cap, tau 0.05, theta 8). */
void cc_default_options(cc_options* opt);

int cc_version(void);

/* Message for the last failing call on this host thread ("" if none). */
const char* cc_last_error(void);

/* Label the components of one graph.
 *  u, v       device, int32[m]: edge i joins u[i] and v[i]; ids in [0, n).
 *             Self-loops and repeated edges are allowed (they change nothing).
 *  m          number of edges, >= 0.
 *  n          number of vertices, >= 0; vertices in no edge get label x.
 *  labels     device, int32[n], written: labels[x] = min id of x's component.
 *  stream     hipStream_t or NULL.
 * Errors: CC_EINVAL (m < 0, n < 0, m > 0 with n == 0, NULL with non-zero size),
 * CC_ERANGE, CC_ENOMEM, CC_EHIP. */
int cc_label(const int32_t* u, const int32_t* v, int64_t m, int32_t n, int32_t* labels, void* stream);

/* cc_label with options (NULL = defaults) and statistics (NULL = not wanted). */
int cc_label_ex(const int32_t* u, const int32_t* v, int64_t m, int32_t n, int32_t* labels, void* stream,
                const cc_options* opt, cc_stats* stats);

/* Arbitrary 64-bit vertex ids (Section III-B relabels the ids of a graph to
 * [0, |V|) before its BFS; Section V treats every id as a 64-bit integer).
 *  u, v       device, int64[m]: edge i joins u[i] and v[i]; any 64-bit value
 *             is an id (INT64_MIN included), repeats and self-loops allowed.
 *  n_max      an upper bound on the number of distinct ids (<= 0: 2m, the
 *             most m edges can have); at most 2^30.  Sizes the device hash
 *             table (2 n_max slots rounded up to a power of two, 8 bytes each)
 *             and bounds the outputs.
 *  ids        device, int64[n_max], written: each distinct id once, in an
 *             unspecified order (it may differ between calls).
 *  labels     device, int64[n_max], written: labels[i] = the smallest id of
 *             the component of ids[i].
 *  n_out      host: the number of distinct ids (entries written).
 * The ids are compacted to [0, n) on the device (hash table + scan), the
 * compact graph is labelled like cc_label (route from opt, as cc_label_ex),
 * and the labels are mapped back to original ids.  Scratch is the cached
 * per-device workspace (calls serialise on it; opt->workspace must be NULL).
 * Errors: CC_EINVAL (m < 0, NULL pointers, n_max above 2^30, more distinct
 * ids than n_max: outputs undefined), CC_ENOMEM, CC_EHIP. */
int cc_label64(const int64_t* u, const int64_t* v, int64_t m, int64_t n_max, int64_t* ids, int64_t* labels,
               int64_t* n_out, void* stream);
int cc_label64_ex(const int64_t* u, const int64_t* v, int64_t m, int64_t n_max, int64_t* ids, int64_t* labels,
                  int64_t* n_out, void* stream, const cc_options* opt, cc_stats* stats);

/* Algorithm 1 as the paper runs it (Section III-A.2, with the sorts of
 * Section III-A.3): the tuple array <p, q, r>, grouped by radix sorts four
 * times per iteration, with the pointer-doubling temporary tuples.  An
 * ablation beside the atomic-hooking SV of cc_label, to measure the share of
 * time the sorts take (Section V, Performance Anatomy).  exclude != 0 sets
 * completed partitions aside as
 * Section III-A.4 describes: after the first join of an iteration, a
 * partition whose vertices are in no other partition, and which did not
 * move, gets its labels and leaves the array.  Same arguments, result and
 * errors as cc_label otherwise (n + 2m + n must stay below 2^32); scratch is
 * the cached per-device workspace, about 32 bytes per tuple.  st (host, may
 * be NULL) receives: */
typedef struct cc_tuple_stats {
    int32_t iterations;       /* iterations of Algorithm 1 until no partition changed */
    int32_t sorts;            /* radix sorts (4 per iteration) */
    int32_t passes_per_sort;  /* 8-bit digit passes of each sort (the key is two ids) */
    int32_t reserved;
    int64_t tuples;           /* n + 2m */
    double ms_sort;           /* device time of the sorts */
    double ms_total;          /* whole call, host clock */
} cc_tuple_stats;
int cc_label_tuples(const int32_t* u, const int32_t* v, int64_t m, int32_t n, int32_t* labels, void* stream,
                    int32_t exclude, cc_tuple_stats* st);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): cc_label on the plain SV
 * route (R1) that allocates nothing, neither device nor host memory.  Its
 * device scratch is a fixed array of CC_NOALLOC_SCRATCH_BYTES inside the
 * library's code object, one copy per GPU, held from load until the process
 * ends; readbacks use the calling thread's stack.  Arguments, outputs,
 * errors and synchrony are those of cc_label.  Limit: m edges need
 * cc_workspace_size(m, n, CC_ROUTE_SV) <= CC_NOALLOC_SCRATCH_BYTES, which
 * holds for every m up to 3 300 000 (any n); a larger m returns CC_EINVAL
 * before any device work.  Every call on one GPU uses that GPU's one array:
 * calls that overlap on one GPU (from several threads or streams) race and
 * must not be made. */
#define CC_NOALLOC_SCRATCH_BYTES (64 * 1024 * 1024)
int cc_label_noalloc(const int32_t* u, const int32_t* v, int64_t m, int32_t n, int32_t* labels, void* stream);

/* Label G independent graphs in one call (one persistent launch for the
 * SV iteration over all of them).
 *  u, v       device, int32: graph g owns edges [edge_off[g], edge_off[g+1]);
 *             ids are graph-local, in [0, n_g) with n_g = vert_off[g+1] - vert_off[g].
 *  edge_off   device, int64[G+1], edge_off[0] = 0, non-decreasing.
 *  vert_off   device, int64[G+1], vert_off[0] = 0, non-decreasing, total < 2^31.
 *  labels     device, int32[vert_off[G]]: graph-local labels (min local id).
 * The launch shape (grid size, hook attempts per pass) is timed over a few
 * candidates on the first call of each size class and remembered; if the
 * environment variable CC_AUTOTUNE_CACHE names a file, the choices are also
 * kept there (one "key blocks link" line per class) and read back on start.
 * If the device refuses the cooperative launch (another process using the
 * same GPU holds its global wave-sync resource), the batch is labelled as one
 * disjoint-union graph by the single-graph SV loop instead: same labels, one
 * host round trip per pass; cc_batch_stats.blocks is then 0.
 * Errors: CC_EINVAL (G < 0, bad offsets: checked on the device), CC_ERANGE,
 * CC_ENOMEM, CC_EHIP, CC_EINTERNAL (the persistent grid's barrier waited more
 * than ~5 s: not every workgroup became resident). */
int cc_label_batched(const int32_t* u, const int32_t* v, const int64_t* edge_off, const int64_t* vert_off,
                     int32_t G, int32_t* labels, void* stream);

/* Batched statistics: passes of the persistent loop and the launch shape used. */
typedef struct cc_batch_stats {
    int32_t passes;      /* SV passes of the persistent loop */
    int32_t tile_edges;  /* edges per workgroup segment */
    int32_t blocks;      /* workgroups of the persistent grid (0: disjoint-union fallback) */
    int32_t max_link;    /* hook attempts per edge per pass */
    int64_t total_edges;
    int64_t total_vertices;
    double ms_total;     /* device time of the launch */
    float pass_ms[32];   /* device time of pass i (the entry after the last pass: final labels) */
    int64_t atomics;           /* atomicMin operations issued, over all passes */
    int64_t chase_reads;       /* parent[] reads of the walks beyond two per active edge */
    int64_t edges_read;        /* active edges read, summed over the passes */
    int64_t survivors_written; /* edges kept for a later pass, summed over the passes */
} cc_batch_stats;

/* cc_label_batched with an explicit launch shape and statistics (may be NULL).
 * tile_edges > 0: about that many edges per workgroup (the grid is rounded to
 * a multiple of 8 and capped at the co-resident maximum); max_link > 0: hook
 * attempts per edge and pass (1 = plain SV).  A zero in either selects the
 * autotuned value, timed on the first call of each size class. */
int cc_label_batched_ex(const int32_t* u, const int32_t* v, const int64_t* edge_off, const int64_t* vert_off,
                        int32_t G, int32_t* labels, void* stream, int32_t tile_edges, int32_t max_link,
                        cc_batch_stats* stats);

/* ------------------------------------------------------------------ router */
/* Number of float32 parameters of the 66 -> 64 -> 64 -> 3 MLP: W1[64][66], b1[64],
 * W2[64][64], b2[64], W3[3][64], b3[3], in that order, row-major [out][in]. */
#define CC_ROUTER_NPARAMS (64 * 66 + 64 + 64 * 64 + 64 + 3 * 64 + 3)
#define CC_ROUTER_NFEATURES 66

/* Load router weights from a text file: CC_ROUTER_NPARAMS decimal floats
 * separated by blanks or line breaks, lines of any length (lines starting
 * with '#' are comments).  Returns CC_EINVAL, keeping the weights loaded
 * before, if the file cannot be read, a token is not a finite number, or the
 * count is wrong. */
int cc_router_load(const char* path);
/* Set router weights from host memory (float32[CC_ROUTER_NPARAMS]); NULL unloads. */
int cc_router_set(const float* host_params);
int cc_router_loaded(void);

/* ---------------------------------------------------------- step entry points
 * The individual steps of the path, exposed so each can be checked on its own.
 * All pointers are device pointers unless marked "host". */

/* Degree (Section III-B, Degree_Distribution): deg[x] = number of edge endpoints
 * equal to x (each undirected edge counts for both ends, a self-loop twice).
 * deg: int32[n], written.  Requires n <= 2^29 (bucketed counting in LDS) and
 * m < 2^31 (else CC_EINVAL).  Returns CC_ERANGE if an id is outside [0, n). */
int cc_degree(const int32_t* u, const int32_t* v, int64_t m, int32_t n, int32_t* deg, void* stream);

/* Degree histograms: hist64[64] (half-octave log bins: bin 0 = degree 0, degree
 * d >= 1 with k = floor(log2 d) goes to 1 + 2k, plus 1 if k >= 1 and bit k-1 of
 * d is set), histx[4096] (exact counts for d < 4096), tail[] (every degree
 * >= 4096, unordered, at most tail_cap written), *tail_count (host, total
 * number of such vertices) and *argmax (host: vertex of maximum degree,
 * smallest id on ties; -1 if n == 0).  hist64/histx are int64 device arrays. */
int cc_degree_histograms(const int32_t* deg, int32_t n, int64_t* hist64, int64_t* histx, int32_t* tail,
                         int64_t tail_cap, int64_t* tail_count, int32_t* argmax, void* stream);

/* Discrete power-law fit and K-S statistic of a degree distribution given as
 * host arrays histx[4096] (counts of degrees below 4096) and tail[ntail] (the
 * degrees >= 4096, any order; CC_EINVAL if one is smaller).
 * Clauset-Shalizi-Newman: for each candidate cutoff d_min
 * (distinct degree with >= 50 vertices and >= 2 distinct values at or above
 * it) alpha is the maximum-likelihood exponent on (1, 10] and D the largest
 * CDF gap; the result is the smallest D (the first such d_min on ties).
 * out (host double[5]): D (+inf if no candidate), alpha, d_min, tail size,
 * candidates.  The candidates are fitted on the current device (one
 * workgroup each, default stream); the call returns when done. */
int cc_powerlaw_ks(const int64_t* histx, const int32_t* tail, int64_t ntail, double* out);

/* CSR of the undirected graph (both directions of every edge, a self-loop
 * twice): off: int64[n+1] = exclusive scan of the degrees; adj: int32[2m]
 * neighbour lists, each vertex's entries in an unspecified order; deg:
 * optional int32[n] output of the degrees (NULL if not wanted).  Requires
 * n <= 2^29 and m < 2^31 (else CC_EINVAL).  Returns CC_ERANGE if an id is
 * outside [0, n). */
int cc_csr(const int32_t* u, const int32_t* v, int64_t m, int32_t n, int32_t* deg, int64_t* off, int32_t* adj,
           void* stream);

/* Direction-optimising BFS from seed over a CSR (off, adj) with n vertices and
 * nadj adjacency entries (checked: off[0] = 0, non-decreasing, off[n] = nadj,
 * entries in [0, n), else CC_EINVAL).
 * visited: uint32[(n+31)/32] bitmap, written (bit x%32 of word x/32).
 * *levels and *bottom_up (host, may be NULL) receive level counts. */
int cc_bfs(const int64_t* off, const int32_t* adj, int32_t n, int64_t nadj, int32_t seed, uint32_t* visited,
           int32_t* levels, int32_t* bottom_up, void* stream);

/* BFS component label and edge filter (Algorithm 2, filter step): labels[x] =
 * min visited id for visited x, x otherwise; (fu, fv) = the edges whose first
 * endpoint is not visited, in an unspecified order; *m_kept and *label (host)
 * receive their count and the component label (-1 if nothing is visited). */
int cc_bfs_filter(const int32_t* u, const int32_t* v, int64_t m, int32_t n, const uint32_t* visited,
                  int32_t* labels, int32_t* fu, int32_t* fv, int64_t* m_kept, int32_t* label, void* stream);

/* Router network on the device: logits[batch][3] for features x[batch][66]
 * (params as in CC_ROUTER_NPARAMS, device float32). */
int cc_mlp_forward(const float* params, const float* x, int32_t batch, float* logits, void* stream);

/* One SGD step of the router on a batch: mean softmax cross-entropy over
 * (x[batch][66], y[batch] in {0,1,2}); params updated in place with step lr;
 * grads (device float32[CC_ROUTER_NPARAMS], may be NULL) receives the gradient;
 * *loss (host, may be NULL) the batch loss before the step. */
int cc_mlp_sgd_step(float* params, const float* x, const int32_t* y, int32_t batch, float lr, float* grads,
                    float* loss, void* stream);

/* Bytes of device scratch a cc_label_ex call on m edges and n vertices may
 * use with this route (CC_ROUTE_*): the size to give cc_options.workspace.
 * The forced SV routes need about 20 bytes per edge; the routes that may
 * take the degree pass and the BFS step about 60 bytes per edge and 40 per
 * vertex.  Negative (CC_EINVAL) for a negative size or a bad route. */
int64_t cc_workspace_size(int64_t m, int32_t n, int32_t route);

/* Trim the current device's scratch pool and free its cached workspace
 * (waits for the device first). */
int cc_release_workspace(void);

/* Free everything the library holds on every device it used: cached
 * workspaces, scratch pools, pinned staging buffers and the router weights'
 * device copies (the loaded weights stay loaded and are copied again on next
 * use).  Waits for those devices first.  No call may be running; later calls
 * work as on first use. */
int cc_shutdown(void);

/* ------------------------------------------------------- measured ceilings */

/* What the device sustains, measured now on `stream` (about a second; it
 * allocates and frees about 6 GiB).  The kernels' rates are compared with
 * these besides the published HBM peak: the SV pass's parent[] gathers and
 * hooks are random 4-byte accesses, its largest-tree probes hit a bitmap in
 * L2, and neither streams. */
typedef struct cc_peaks {
    double copy_gbps;          /* streaming 16-byte copy of 1 GiB: bytes read + written per second / 1e9
                                  (best of a plain, a 4-in-flight and a non-temporal form) */
    double copy_bytes;         /* bytes moved per copy launch (read + written) */
    double read_gbps;          /* streaming read of 1 GiB (best of a plain and a non-temporal form) */
    int64_t table_bytes[3];    /* table sizes: 2 MiB (fits one XCD's L2), 64 MiB (Infinity Cache), 4 GiB (HBM) */
    double gather_gps[3];      /* random 4-byte loads per second / 1e9, per table */
    double atomic_gps[3];      /* random agent-scope atomicMin with the old value returned, per second / 1e9 */
    double accesses;           /* random accesses per launch (8 in flight per thread) */
} cc_peaks;
/* Errors: CC_EINVAL (NULL out), CC_ENOMEM, CC_EHIP.  Best of five launches
 * after a warm-up for each figure. */
int cc_measure_peaks(cc_peaks* out, void* stream);

/* ------------------------------------------------------------ checking */

/* Checks a labelling on the device against the invariants every exact
 * result meets: I1, the two ends of each edge carry the same label, and
 * I2, labels[x] <= x and labels[labels[x]] == labels[x].  They hold for the
 * component-minimum labelling, and any labelling that breaks one is wrong;
 * a labelling that merged two components into one can still pass (only a
 * comparison with the exact result sees that).
 *  u, v, m, n as for cc_label; labels device int32[n], read only.
 *  bad        host int64[3], written: edges whose ends carry different
 *             labels, vertices breaking I2, edges with an end outside [0, n).
 * Returns CC_OK whatever the counts (they are the result); CC_EINVAL for bad
 * arguments, CC_EHIP.  Uses the cached per-device workspace. */
int cc_check_labels(const int32_t* u, const int32_t* v, int64_t m, int32_t n, const int32_t* labels, void* stream,
                    int64_t* bad);

/* Test hook for the failure paths: the nth device or pinned-host allocation
 * the library makes from now on (workspace growth, pool allocation, pinned
 * staging, router copies) fails as if memory were exhausted, so the call
 * making it returns CC_ENOMEM; the count is process-wide and fires once.
 * nth = 0 turns a pending failure off.  Returns CC_OK, or CC_EINVAL for
 * nth < 0.  A call that failed this way leaves the library usable: the next
 * call allocates afresh.  The environment variable CCMI_FAIL_ALLOC=k arms
 * the same countdown once, at the process's first allocation. */
int cc_debug_fail_alloc(int64_t nth);

#ifdef __cplusplus
}
#endif

#endif /* CCMI_CC_H */
