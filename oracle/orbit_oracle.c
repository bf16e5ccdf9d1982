/*
 * orbit_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct CPU reference for per-vertex graphlet
 * orbit counts (all connected patterns with 2..5 vertices, orbits 0-72).
 * Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load it; the GPU library never does, and the two share
 * no code, tables or generators.
 *
 * What it computes, straight from the definitions in the paper:
 *   - Definition "auto" (Preliminaries): orbits are the classes of the
 *     automorphism relation on the vertices of a pattern.  The patterns
 *     H0..H29 and the label of one vertex of every orbit are transcribed
 *     from the figure of all vertex orbits (Fig. node_orbits); the orbit
 *     of every other vertex is derived by computing automorphisms.
 *   - Induced orbit counts (Introduction, "Problem Description"; and the
 *     induced/non-induced paragraph of the Preliminaries): for vertex u and
 *     orbit theta of a k-vertex pattern H, the number of k-subsets S
 *     containing u with G[S] isomorphic to H and u mapped into theta.
 *     Obtained by visiting every connected induced k-subset (k=2..5) once,
 *     with the ESU enumeration of Wernicke (2006), and looking the
 *     subset's labelled adjacency bitmask up in a table built by trying
 *     every permutation of every pattern.
 *   - Non-induced counts DM(u, theta) (Definition "unlabeled-match"): the
 *     number of distinct non-induced copies (vertex set + edge subset)
 *     isomorphic to H with u in theta.  Every such copy lives inside one
 *     connected vertex subset; for each subset every connected spanning
 *     edge subset is classified with the same table.
 *   - Rooted counts: induced counts of one vertex only, enumerating the
 *     connected subsets that contain it, with an optional subset budget.
 *   - Edge orbit counts E_0..E_11 (Definition edge-orbit; the matches of
 *     an edge orbit in the definition after Fig. edge_orbits): edge
 *     orbits are the classes of the automorphism relation on the edges of
 *     the 3- and 4-vertex patterns, labelled from Fig. edge_orbits; every
 *     non-induced copy of such a pattern (a connected spanning edge subset
 *     of a connected 3- or 4-subset) adds one to each of its edges, at the
 *     slot (u,v) whose u lies in the endpoint orbit of larger index, and
 *     at both slots when the two endpoint orbits are the same.
 *
 * All counts are uint64 and wrap modulo 2^64.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#include <pthread.h>
#endif

#define NORB 73
#define NGRAPHLET 30
#define MAXK 5

/* ---- pattern transcription (Fig. node_orbits) ---------------------------
 * Each pattern: number of vertices, edge list on 1-based TikZ node ids, and
 * (node, printed orbit label) for every labelled node in the figure.      */
typedef struct {
    int k;
    int ne;
    int e[10][2];
    int nl;
    int lab[5][2];
} pattern_t;

static const pattern_t PATTERNS[NGRAPHLET] = {
    /* H0 */ {2, 1, {{1,2}}, 1, {{2,0}}},
    /* H1 */ {3, 2, {{1,2},{2,3}}, 2, {{2,2},{3,1}}},
    /* H2 */ {3, 3, {{1,2},{1,3},{2,3}}, 1, {{3,3}}},
    /* H3 */ {4, 3, {{1,2},{2,3},{3,4}}, 2, {{3,5},{4,4}}},
    /* H4 */ {4, 3, {{1,3},{2,3},{3,4}}, 2, {{3,7},{4,6}}},
    /* H5 */ {4, 4, {{1,2},{1,3},{2,4},{3,4}}, 1, {{3,8}}},
    /* H6 */ {4, 4, {{1,2},{2,3},{2,4},{3,4}}, 3, {{1,9},{2,11},{3,10}}},
    /* H7 */ {4, 5, {{1,2},{1,3},{1,4},{2,4},{3,4}}, 2, {{2,12},{4,13}}},
    /* H8 */ {4, 6, {{1,2},{1,3},{1,4},{2,3},{2,4},{3,4}}, 1, {{4,14}}},
    /* H9 */ {5, 4, {{1,2},{2,3},{3,4},{4,5}}, 3, {{3,17},{4,16},{5,15}}},
    /* H10 */ {5, 4, {{1,3},{2,3},{3,4},{4,5}}, 4, {{1,19},{3,21},{4,20},{5,18}}},
    /* H11 */ {5, 4, {{1,3},{2,3},{3,4},{3,5}}, 2, {{3,23},{5,22}}},
    /* H12 */ {5, 5, {{1,3},{2,4},{3,4},{3,5},{4,5}}, 3, {{1,24},{3,26},{5,25}}},
    /* H13 */ {5, 5, {{1,2},{1,3},{2,3},{3,4},{4,5}}, 4, {{1,29},{3,30},{4,28},{5,27}}},
    /* H14 */ {5, 5, {{1,3},{2,3},{3,4},{3,5},{4,5}}, 3, {{1,31},{3,33},{4,32}}},
    /* H15 */ {5, 5, {{1,2},{1,3},{2,4},{3,5},{4,5}}, 1, {{5,34}}},
    /* H16 */ {5, 5, {{1,2},{2,3},{2,4},{3,5},{4,5}}, 4, {{1,35},{2,38},{3,37},{5,36}}},
    /* H17 */ {5, 6, {{1,2},{2,3},{2,4},{2,5},{3,5},{4,5}}, 4, {{1,39},{2,42},{3,40},{5,41}}},
    /* H18 */ {5, 6, {{1,2},{1,3},{2,3},{3,4},{3,5},{4,5}}, 2, {{3,44},{4,43}}},
    /* H19 */ {5, 6, {{1,2},{2,3},{2,4},{3,4},{3,5},{4,5}}, 4, {{1,45},{2,47},{3,48},{5,46}}},
    /* H20 */ {5, 6, {{1,2},{1,3},{1,4},{2,5},{3,5},{4,5}}, 2, {{1,50},{2,49}}},
    /* H21 */ {5, 6, {{1,2},{1,3},{2,4},{3,4},{3,5},{4,5}}, 3, {{1,51},{3,53},{5,52}}},
    /* H22 */ {5, 7, {{1,3},{1,4},{2,3},{2,4},{3,4},{3,5},{4,5}}, 2, {{1,54},{3,55}}},
    /* H23 */ {5, 7, {{1,2},{2,3},{2,4},{2,5},{3,4},{3,5},{4,5}}, 3, {{1,56},{2,58},{3,57}}},
    /* H24 */ {5, 7, {{1,2},{1,3},{2,3},{2,4},{3,4},{3,5},{4,5}}, 3, {{1,59},{2,60},{3,61}}},
    /* H25 */ {5, 7, {{1,2},{1,3},{1,4},{2,5},{3,4},{3,5},{4,5}}, 3, {{2,62},{3,64},{5,63}}},
    /* H26 */ {5, 8, {{1,2},{1,3},{2,3},{2,4},{2,5},{3,4},{3,5},{4,5}}, 3, {{1,65},{3,67},{5,66}}},
    /* H27 */ {5, 8, {{1,2},{1,3},{1,4},{2,3},{2,5},{3,4},{3,5},{4,5}}, 2, {{3,69},{4,68}}},
    /* H28 */ {5, 9, {{1,2},{1,3},{1,4},{2,3},{2,4},{2,5},{3,4},{3,5},{4,5}}, 2, {{1,70},{4,71}}},
    /* H29 */ {5, 10, {{1,2},{1,3},{1,4},{1,5},{2,3},{2,4},{2,5},{3,4},{3,5},{4,5}}, 1, {{5,72}}},
};

/* ---- edge orbit transcription (Fig. edge_orbits) --------------------------
 * For each printed edge-orbit label 0..11: the pattern and the TikZ node ids
 * of the edge the label is drawn beside.  The figure's drawings of H1..H8
 * number their nodes as the figure of vertex orbits does.                  */
#define NEORB 12
static const int EDGE_LABELS[NEORB][3] = {
    /* label: pattern, node, node */
    {1, 2, 3}, {2, 1, 3}, {3, 3, 4}, {3, 2, 3}, {4, 3, 4}, {5, 3, 4},
    {6, 1, 2}, {6, 3, 4}, {6, 2, 4}, {7, 2, 4}, {7, 1, 4}, {8, 1, 4},
};

/* ---- derived tables ---------------------------------------------------- */
static int g_status = 0;               /* 0 ok; <0 transcription inconsistent */
static int g_node_orbit[NGRAPHLET][MAXK];
static int g_aut[NGRAPHLET];
static int g_orbit_graphlet[NORB];
static int g_orbit_size[NORB];
/* pair index of (i,j), i<j, positions 0..4 */
static int g_pair[MAXK][MAXK];
/* LUT per k: graphlet id (or -1 if disconnected) and orbit of each position */
static signed char g_lut_graphlet[MAXK + 1][1024];
static signed char g_lut_orbit[MAXK + 1][1024][MAXK];
/* edge orbit of an edge whose endpoints lie in vertex orbits (hi, lo),
 * hi >= lo, of a 3- or 4-vertex pattern; -1 if no edge orbit has them */
static signed char g_edge_label[15][15];

static int next_perm(int *a, int k) {
    int i = k - 2;
    while (i >= 0 && a[i] >= a[i + 1]) i--;
    if (i < 0) return 0;
    int j = k - 1;
    while (a[j] <= a[i]) j--;
    int t = a[i]; a[i] = a[j]; a[j] = t;
    for (int l = i + 1, r = k - 1; l < r; l++, r--) { t = a[l]; a[l] = a[r]; a[r] = t; }
    return 1;
}

static int pattern_mask(const pattern_t *p, const int *pos_of_node) {
    int mask = 0;
    for (int e = 0; e < p->ne; e++) {
        int x = pos_of_node[p->e[e][0] - 1], y = pos_of_node[p->e[e][1] - 1];
        int lo = x < y ? x : y, hi = x < y ? y : x;
        mask |= 1 << g_pair[lo][hi];
    }
    return mask;
}

/* Edge orbits of patterns H1..H8: classes of edges under the automorphisms
 * (permutations preserving the edge set), each labelled from the figure;
 * then the (endpoint orbit, endpoint orbit) -> label table, which must be
 * unambiguous for the classification by vertex orbits to be valid. */
static void build_edge_tables(void) {
    memset(g_edge_label, -1, sizeof g_edge_label);
    for (int h = 1; h <= 8; h++) {
        const pattern_t *p = &PATTERNS[h];
        int k = p->k;
        int base = pattern_mask(p, (int[]){0, 1, 2, 3, 4});
        int cls[10];  /* class of each pattern edge (index into p->e) */
        for (int e = 0; e < p->ne; e++) cls[e] = e;
        int perm[MAXK] = {0, 1, 2, 3, 4};
        do {
            if (pattern_mask(p, perm) != base) continue;
            for (int e = 0; e < p->ne; e++) {
                int x = perm[p->e[e][0] - 1], y = perm[p->e[e][1] - 1];
                for (int f = 0; f < p->ne; f++) {
                    int a = p->e[f][0] - 1, b = p->e[f][1] - 1;
                    if ((a == x && b == y) || (a == y && b == x)) {
                        int c1 = cls[e], c2 = cls[f];
                        int lo = c1 < c2 ? c1 : c2, hi = c1 < c2 ? c2 : c1;
                        for (int g = 0; g < p->ne; g++) if (cls[g] == hi) cls[g] = lo;
                    }
                }
            }
        } while (next_perm(perm, k));
        int label_of_class[10];
        for (int e = 0; e < p->ne; e++) label_of_class[e] = -1;
        for (int l = 0; l < NEORB; l++) {
            if (EDGE_LABELS[l][0] != h) continue;
            int a = EDGE_LABELS[l][1], b = EDGE_LABELS[l][2], found = -1;
            for (int e = 0; e < p->ne; e++)
                if ((p->e[e][0] == a && p->e[e][1] == b) || (p->e[e][0] == b && p->e[e][1] == a))
                    found = e;
            if (found < 0) { g_status = -7; continue; }
            if (label_of_class[cls[found]] != -1) g_status = -8;
            label_of_class[cls[found]] = l;
        }
        for (int e = 0; e < p->ne; e++) {
            int l = label_of_class[cls[e]];
            if (l < 0) { g_status = -9; continue; }
            int oa = g_node_orbit[h][p->e[e][0] - 1], ob = g_node_orbit[h][p->e[e][1] - 1];
            int hi = oa > ob ? oa : ob, lo = oa > ob ? ob : oa;
            if (g_edge_label[hi][lo] != -1 && g_edge_label[hi][lo] != l) g_status = -10;
            g_edge_label[hi][lo] = (signed char)l;
        }
    }
}

static void build_tables(void) {
    /* pairs ordered by their larger element, so that a k-vertex mask uses
       exactly bits 0..C(k,2)-1 */
    int idx = 0;
    for (int j = 1; j < MAXK; j++)
        for (int i = 0; i < j; i++) g_pair[i][j] = g_pair[j][i] = idx++;

    memset(g_lut_graphlet, -1, sizeof g_lut_graphlet);
    memset(g_lut_orbit, -1, sizeof g_lut_orbit);
    for (int o = 0; o < NORB; o++) { g_orbit_graphlet[o] = -1; g_orbit_size[o] = 0; }

    for (int h = 0; h < NGRAPHLET; h++) {
        const pattern_t *p = &PATTERNS[h];
        int k = p->k;
        int base = pattern_mask(p, (int[]){0, 1, 2, 3, 4});
        /* automorphisms: permutations that preserve the edge mask */
        int cls[MAXK];
        for (int i = 0; i < k; i++) cls[i] = i;
        int perm[MAXK] = {0, 1, 2, 3, 4};
        int aut = 0;
        do {
            if (pattern_mask(p, perm) == base) {
                aut++;
                /* union node x with perm[x] */
                for (int x = 0; x < k; x++) {
                    int a = cls[x], b = cls[perm[x]];
                    if (a != b) {
                        int lo = a < b ? a : b, hi = a < b ? b : a;
                        for (int y = 0; y < k; y++) if (cls[y] == hi) cls[y] = lo;
                    }
                }
            }
        } while (next_perm(perm, k));
        g_aut[h] = aut;
        /* label every class from its labelled node; exactly one label per class */
        int label_of_class[MAXK];
        for (int i = 0; i < k; i++) label_of_class[i] = -1;
        for (int l = 0; l < p->nl; l++) {
            int c = cls[p->lab[l][0] - 1];
            if (label_of_class[c] != -1) g_status = -1;
            label_of_class[c] = p->lab[l][1];
        }
        for (int x = 0; x < k; x++) {
            int o = label_of_class[cls[x]];
            if (o < 0) { g_status = -2; o = 0; }
            g_node_orbit[h][x] = o;
            if (g_orbit_graphlet[o] != -1 && g_orbit_graphlet[o] != h) g_status = -3;
            g_orbit_graphlet[o] = h;
            g_orbit_size[o]++;
        }
        /* LUT: every relabelling of the pattern onto positions 0..k-1 */
        int pos[MAXK] = {0, 1, 2, 3, 4};
        do {
            int mask = pattern_mask(p, pos);
            if (g_lut_graphlet[k][mask] != -1 && g_lut_graphlet[k][mask] != h) g_status = -4;
            g_lut_graphlet[k][mask] = (signed char)h;
            for (int x = 0; x < k; x++) {
                int o = g_node_orbit[h][x];
                if (g_lut_orbit[k][mask][pos[x]] != -1 && g_lut_orbit[k][mask][pos[x]] != o) g_status = -5;
                g_lut_orbit[k][mask][pos[x]] = (signed char)o;
            }
        } while (next_perm(pos, k));
    }
    for (int o = 0; o < NORB; o++) if (g_orbit_graphlet[o] < 0) g_status = -6;
    build_edge_tables();
}

/* The tables are built once, also when several host threads make their
 * first call at the same time. */
static pthread_once_t g_once = PTHREAD_ONCE_INIT;
static void ensure_tables(void) {
    pthread_once(&g_once, build_tables);
}

/* ---- graph access ------------------------------------------------------ */
typedef struct {
    const uint32_t *rp;
    const uint32_t *ci;
    uint32_t n;
} graph_t;

static int adjacent(const graph_t *g, uint32_t u, uint32_t v) {
    uint32_t lo = g->rp[u], hi = g->rp[u + 1];
    while (lo < hi) {
        uint32_t mid = lo + (hi - lo) / 2;
        if (g->ci[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo < g->rp[u + 1] && g->ci[lo] == v;
}

/* induced adjacency bitmask of the positions 0..k-1 of set s */
static int set_mask(const graph_t *g, const uint32_t *s, int k) {
    int mask = 0;
    for (int j = 1; j < k; j++)
        for (int i = 0; i < j; i++)
            if (adjacent(g, s[i], s[j])) mask |= 1 << g_pair[i][j];
    return mask;
}

/* ---- ESU enumeration ----------------------------------------------------
 * Visits every connected vertex subset of size 2..kmax that contains the
 * root and in which the root has the smallest key, exactly once.  The key
 * of a vertex is its id, except that the root's own key is taken as -1
 * when `root_first` is set (then every connected subset containing the
 * root is visited).                                                        */
typedef struct {
    const graph_t *g;
    int kmax;
    uint32_t root;
    int root_first;
    int noninduced;
    uint64_t *counts;          /* n x 73 (full mode) or 73 (rooted mode) */
    int rooted;
    uint64_t budget;           /* 0 = unlimited */
    uint64_t visited;
    int exhausted;
    uint64_t *ecounts;         /* non-induced mode: 2m x 12 edge orbit counts, or NULL */
    int eerr;                  /* an edge whose endpoint orbits name no edge orbit */
} esu_t;

/* slot of v in the neighbour list of u (v must be a neighbour) */
static uint64_t slot_of(const graph_t *g, uint32_t u, uint32_t v) {
    uint32_t lo = g->rp[u], hi = g->rp[u + 1];
    while (lo < hi) {
        uint32_t mid = lo + (hi - lo) / 2;
        if (g->ci[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo;
}

/* one non-induced copy (edge mask sub of positions 0..k-1 of s, pattern of
 * 3 or 4 vertices): one count for every edge, at its oriented slot(s) */
static void count_copy_edges(esu_t *st, const uint32_t *s, int k, int sub) {
    for (int j = 1; j < k; j++)
        for (int i = 0; i < j; i++) {
            if (!(sub >> g_pair[i][j] & 1)) continue;
            int oi = g_lut_orbit[k][sub][i], oj = g_lut_orbit[k][sub][j];
            int hi = oi > oj ? oi : oj, lo = oi > oj ? oj : oi;
            int l = (hi < 15) ? g_edge_label[hi][lo] : -1;
            if (l < 0) { st->eerr = 1; continue; }
            if (oi >= oj) st->ecounts[slot_of(st->g, s[i], s[j]) * NEORB + l]++;
            if (oj >= oi) st->ecounts[slot_of(st->g, s[j], s[i]) * NEORB + l]++;
        }
}

static int64_t key_of(const esu_t *st, uint32_t v) {
    return (st->root_first && v == st->root) ? -1 : (int64_t)v;
}

static void classify(esu_t *st, const uint32_t *s, int k) {
    int mask = set_mask(st->g, s, k);
    if (!st->noninduced) {
        if (g_lut_graphlet[k][mask] < 0) return; /* cannot happen: s is connected */
        if (st->rooted) {
            for (int i = 0; i < k; i++)
                if (s[i] == st->root) st->counts[g_lut_orbit[k][mask][i]]++;
        } else {
            for (int i = 0; i < k; i++)
                st->counts[(uint64_t)s[i] * NORB + g_lut_orbit[k][mask][i]]++;
        }
        return;
    }
    /* non-induced: every connected spanning edge subset of G[s] */
    for (int sub = mask;; sub = (sub - 1) & mask) {
        if (g_lut_graphlet[k][sub] >= 0 && st->ecounts && k >= 3 && k <= 4)
            count_copy_edges(st, s, k, sub);
        if (g_lut_graphlet[k][sub] >= 0 && st->counts) {
            if (st->rooted) {
                for (int i = 0; i < k; i++)
                    if (s[i] == st->root) st->counts[g_lut_orbit[k][sub][i]]++;
            } else {
                for (int i = 0; i < k; i++)
                    st->counts[(uint64_t)s[i] * NORB + g_lut_orbit[k][sub][i]]++;
            }
        }
        if (sub == 0) break;
    }
}

/* is v in the closed neighbourhood of the current subset? */
static int in_closed_nbhd(const esu_t *st, const uint32_t *s, int k, uint32_t v) {
    for (int i = 0; i < k; i++)
        if (s[i] == v || adjacent(st->g, s[i], v)) return 1;
    return 0;
}

static void esu_extend(esu_t *st, uint32_t *s, int k, const uint32_t *ext, int next) {
    if (st->exhausted) return;
    if (k >= 2) {
        if (st->budget && st->visited >= st->budget) { st->exhausted = 1; return; }
        st->visited++;
        classify(st, s, k);
    }
    if (k == st->kmax) return;
    /* local copy because the extension set shrinks as we iterate */
    uint32_t *work = NULL;
    uint32_t local[256];
    int cap = next;
    if (cap <= 256) work = local;
    else work = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)cap);
    memcpy(work, ext, sizeof(uint32_t) * (size_t)next);
    int nw = next;
    while (nw > 0) {
        uint32_t w = work[--nw];
        /* new extension: remaining work + exclusive neighbours of w */
        const graph_t *g = st->g;
        uint32_t dw = g->rp[w + 1] - g->rp[w];
        size_t newcap = (size_t)nw + dw;
        uint32_t *next_ext = (uint32_t *)malloc(sizeof(uint32_t) * (newcap ? newcap : 1));
        memcpy(next_ext, work, sizeof(uint32_t) * (size_t)nw);
        int nn = nw;
        for (uint32_t p = g->rp[w]; p < g->rp[w + 1]; p++) {
            uint32_t u = g->ci[p];
            if (key_of(st, u) <= key_of(st, st->root)) continue;
            /* exclusive neighbours only: u must not be in, or adjacent to,
               the current subset.  Every vertex still in the extension set
               is adjacent to the subset, so u cannot already be there. */
            if (in_closed_nbhd(st, s, k, u)) continue;
            next_ext[nn++] = u;
        }
        s[k] = w;
        esu_extend(st, s, k + 1, next_ext, nn);
        free(next_ext);
        if (st->exhausted) break;
    }
    if (work != local) free(work);
}

static void esu_root(esu_t *st) {
    const graph_t *g = st->g;
    uint32_t v = st->root;
    uint32_t s[MAXK];
    s[0] = v;
    uint32_t dv = g->rp[v + 1] - g->rp[v];
    uint32_t *ext = (uint32_t *)malloc(sizeof(uint32_t) * (dv ? dv : 1));
    int ne = 0;
    for (uint32_t p = g->rp[v]; p < g->rp[v + 1]; p++) {
        uint32_t u = g->ci[p];
        if (key_of(st, u) > key_of(st, v)) ext[ne++] = u;
    }
    esu_extend(st, s, 1, ext, ne);
    free(ext);
}

/* ---- exported API ------------------------------------------------------ */

/* 0 if the transcribed patterns give 73 orbits with one printed label per
 * automorphism class; negative otherwise. */
int oracle_tables_status(void) {
    ensure_tables();
    return g_status;
}

/* node_orbit[h*5 + x] = orbit of node x+1 of pattern h (-1 past k);
 * aut[h] = |Aut(H_h)|; orbit_graphlet[o]; orbit_size[o]; pattern_k[h]. */
void oracle_tables(int *node_orbit, int *aut, int *orbit_graphlet, int *orbit_size, int *pattern_k) {
    ensure_tables();
    for (int h = 0; h < NGRAPHLET; h++) {
        for (int x = 0; x < MAXK; x++)
            node_orbit[h * MAXK + x] = x < PATTERNS[h].k ? g_node_orbit[h][x] : -1;
        aut[h] = g_aut[h];
        pattern_k[h] = PATTERNS[h].k;
    }
    for (int o = 0; o < NORB; o++) {
        orbit_graphlet[o] = g_orbit_graphlet[o];
        orbit_size[o] = g_orbit_size[o];
    }
}

/* graphlet id of a labelled k-vertex adjacency mask (-1 if disconnected) and
 * the orbit of each of its k positions. */
int oracle_classify_mask(int k, int mask, int *orbit_out) {
    ensure_tables();
    if (k < 2 || k > MAXK || mask < 0 || mask >= (1 << (k * (k - 1) / 2))) return -2;
    for (int i = 0; i < k; i++) orbit_out[i] = g_lut_orbit[k][mask][i];
    return g_lut_graphlet[k][mask];
}

/* pair bit index used by masks (positions i != j, both < 5) */
int oracle_pair_index(int i, int j) {
    ensure_tables();
    return g_pair[i][j];
}

static int full_counts(const uint32_t *rp, const uint32_t *ci, uint32_t n, int kmax,
                       int noninduced, uint64_t *counts, int nthreads) {
    ensure_tables();
    if (g_status) return g_status;
    if (kmax < 2 || kmax > MAXK) return -10;
    graph_t g = {rp, ci, n};
    memset(counts, 0, sizeof(uint64_t) * (size_t)n * NORB);
    int nt = nthreads > 0 ? nthreads : 1;
#ifndef _OPENMP
    nt = 1;
#endif
    if (nt == 1) {
        for (uint32_t v = 0; v < n; v++) {
            esu_t st = {&g, kmax, v, 0, noninduced, counts, 0, 0, 0, 0};
            esu_root(&st);
        }
        return 0;
    }
#ifdef _OPENMP
    /* one private count array per thread, summed at the end */
    uint64_t *part = (uint64_t *)calloc((size_t)nt * n * NORB, sizeof(uint64_t));
    if (!part) return -11;
#pragma omp parallel num_threads(nt)
    {
        int t = omp_get_thread_num();
        uint64_t *mine = part + (size_t)t * n * NORB;
#pragma omp for schedule(dynamic, 16)
        for (int64_t v = 0; v < (int64_t)n; v++) {
            esu_t st = {&g, kmax, (uint32_t)v, 0, noninduced, mine, 0, 0, 0, 0};
            esu_root(&st);
        }
    }
    for (int t = 0; t < nt; t++) {
        uint64_t *mine = part + (size_t)t * n * NORB;
        for (size_t i = 0; i < (size_t)n * NORB; i++) counts[i] += mine[i];
    }
    free(part);
#endif
    return 0;
}

/* Induced orbit counts of every vertex, patterns of 2..kmax vertices. */
int oracle_induced_counts(const uint32_t *rp, const uint32_t *ci, uint32_t n, int kmax,
                          uint64_t *counts, int nthreads) {
    return full_counts(rp, ci, n, kmax, 0, counts, nthreads);
}

/* Non-induced orbit counts DM(u, theta) of every vertex. */
int oracle_noninduced_counts(const uint32_t *rp, const uint32_t *ci, uint32_t n, int kmax,
                             uint64_t *counts, int nthreads) {
    return full_counts(rp, ci, n, kmax, 1, counts, nthreads);
}

/* Induced counts of the listed roots only: counts[r*73 + o].  A root whose
 * enumeration would visit more than `budget` subsets (0 = no limit) gets
 * complete[r] = 0 and its row is partial; otherwise complete[r] = 1. */
int oracle_rooted_counts(const uint32_t *rp, const uint32_t *ci, uint32_t n, int kmax,
                         const uint32_t *roots, uint32_t nroots, uint64_t budget,
                         uint64_t *counts, uint8_t *complete, int nthreads) {
    ensure_tables();
    if (g_status) return g_status;
    if (kmax < 2 || kmax > MAXK) return -10;
    graph_t g = {rp, ci, n};
    memset(counts, 0, sizeof(uint64_t) * (size_t)nroots * NORB);
    int nt = nthreads > 0 ? nthreads : 1;
    (void)nt;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
#endif
    for (int64_t r = 0; r < (int64_t)nroots; r++) {
        if (roots[r] >= n) { complete[r] = 0; continue; }
        esu_t st = {&g, kmax, roots[r], 1, 0, counts + (size_t)r * NORB, 1, budget, 0, 0};
        esu_root(&st);
        complete[r] = st.exhausted ? 0 : 1;
    }
    return 0;
}

/* Non-induced edge orbit counts E_0..E_11 of every slot of the CSR:
 * ecounts[slot * 12 + i] = E_i<u,v> for slot (u,v), u the endpoint in the
 * orbit of larger index (both slots hold E_i when the endpoint orbits are
 * equal).  Returns -12 if a copy has an edge no edge orbit describes. */
int oracle_edge_counts(const uint32_t *rp, const uint32_t *ci, uint32_t n, uint64_t *ecounts,
                       int nthreads) {
    ensure_tables();
    if (g_status) return g_status;
    graph_t g = {rp, ci, n};
    const size_t len = (size_t)rp[n] * NEORB;
    memset(ecounts, 0, sizeof(uint64_t) * len);
    int nt = nthreads > 0 ? nthreads : 1;
    int err = 0;
#ifndef _OPENMP
    nt = 1;
#endif
    if (nt == 1) {
        for (uint32_t v = 0; v < n; v++) {
            esu_t st = {&g, 4, v, 0, 1, NULL, 0, 0, 0, 0, ecounts, 0};
            esu_root(&st);
            err |= st.eerr;
        }
        return err ? -12 : 0;
    }
#ifdef _OPENMP
    uint64_t *part = (uint64_t *)calloc((size_t)nt * len + 1, sizeof(uint64_t));
    if (!part) return -11;
#pragma omp parallel num_threads(nt) reduction(| : err)
    {
        uint64_t *mine = part + (size_t)omp_get_thread_num() * len;
#pragma omp for schedule(dynamic, 16)
        for (int64_t v = 0; v < (int64_t)n; v++) {
            esu_t st = {&g, 4, (uint32_t)v, 0, 1, NULL, 0, 0, 0, 0, mine, 0};
            esu_root(&st);
            err |= st.eerr;
        }
    }
    for (int t = 0; t < nt; t++)
        for (size_t i = 0; i < len; i++) ecounts[i] += part[(size_t)t * len + i];
    free(part);
#endif
    return err ? -12 : 0;
}
