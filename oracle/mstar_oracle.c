/*
 * mstar_oracle.c -- plain, slow, FP64 CPU oracle of the MSTAR algorithmically
 * regularised integrator (Rantala, Pihajoki, Mannerkoski, Johansson & Naab
 * 2020, "MSTAR - a fast parallelised algorithmically regularised integrator
 * with minimum spanning tree coordinates").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference that the GPU library
 * is checked against.  It is used by tests/, by __graft_entry__.smoke() and by
 * bench.py's cpu_baseline leg, and by nothing else; the product library never
 * links or calls it, and it shares no code with the product library.
 *
 * Arithmetic: IEEE-754 binary64, round to nearest even, compiled with
 * -ffp-contract=off and without fast-math, so every +,-,*,/ and sqrt below is
 * one correctly rounded operation in the order written.  OpenMP, where used,
 * parallelises over independent i (each a_i is still summed by one thread in
 * ascending j), so results are bit-identical for any thread count.
 *
 * Each function names the passage of the paper it follows.  Readings taken
 * where the paper is silent are marked READING.  Parity unpinned against the
 * paper (no printed value or closed form fixes them; they are checked
 * oracle-vs-GPU only): the step-controller constants a_GBS, f_min, f_max and
 * the first-step factor q, and the TTL weights omega_ij.  The error measure
 * and the rule that gives a new MST edge its vector at a rebuild are pinned by
 * the CPU tests (closed-form Kepler errors; persisting edges keep their bits).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_E_INVAL -1
#define ORC_E_NOMEM -2
#define ORC_E_NONFINITE -4
#define ORC_E_COINCIDENT -5
#define ORC_E_NOCONV -6
#define ORC_E_MAXSTEPS -7
#define ORC_W_TIME_TOL 1

/* Parameters of the method (Sec. 2.1 triplet, Sec. 2.3 GBS, Sec. 2.4 time
 * iteration, Sec. 3.4 N_d, Sec. 4.2 k_fix).  Layout mirrored by oracle/__init__.py. */
typedef struct {
    double G;
    double eta;            /* GBS tolerance eta_GBS, eq. gbs-criterion */
    double alpha, beta, gamma; /* time-transformation triplet, eq. ttl */
    double omega_mass_max; /* READING: Omega couples only bodies with m <= this */
    double a_gbs, f_min, f_max; /* eq. hnext safety factor and READING clamps */
    double q_first;        /* Sec. 2.4 first-step safety factor */
    double t_tol;          /* relative end-time tolerance */
    double h_init;         /* >0: first fictitious step; 0: automatic */
    int64_t max_steps;
    int32_t k_fix;         /* number of substep divisions, n_k = 2k */
    int32_t n_d;           /* MST closeness N_d, eq. LCA */
    int32_t max_halvings;
    int32_t max_time_iter;
    int32_t rebuild_every; /* accepted steps between MST rebuilds */
    int32_t nthreads;      /* OpenMP threads for the force loop (0 = default) */
    int32_t accept_rule;   /* READING of eq. gbs-criterion vs Sec. 4.2: 0 judge at k_fix;
                              1 accept at the first k >= 2 whose eps_k <= eta */
    int32_t mst_method;    /* 0: exact MST (Sec. 3.2); 1: divide-and-conquer tree (Sec. 3.3) */
} orc_params;

typedef struct {
    int64_t steps_accepted, steps_rejected, force_evals, mst_rebuilds, topo_changes, time_iters;
    double t_reached, eps_last, h_next, h_last;
} orc_stats;

/* ------------------------------------------------------------------ */
/* Neumaier compensated summation (Neumaier 1974; Sec. 3.5 mentions it). */
typedef struct { double s, c; } nsum;
static void ns_init(nsum *a) { a->s = 0.0; a->c = 0.0; }
static void ns_add(nsum *a, double x) {
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}
static double ns_get(const nsum *a) { return a->s + a->c; }

/* ------------------------------------------------------------------ */
/* Centre of mass of a set of vectors, Neumaier sums in index order. */
static void com3(int n, const double *m, const double *x, double out[3]) {
    nsum M, s[3];
    ns_init(&M);
    for (int k = 0; k < 3; ++k) ns_init(&s[k]);
    for (int i = 0; i < n; ++i) {
        ns_add(&M, m[i]);
        for (int k = 0; k < 3; ++k) ns_add(&s[k], m[i] * x[3 * i + k]);
    }
    double Mt = ns_get(&M);
    for (int k = 0; k < 3; ++k) out[k] = ns_get(&s[k]) / Mt;
}

/* The same with plain sums in index order (no compensation). */
static void com3_plain(int n, const double *m, const double *x, double out[3]) {
    double M = 0.0, s[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < n; ++i) {
        M = M + m[i];
        for (int k = 0; k < 3; ++k) s[k] = s[k] + m[i] * x[3 * i + k];
    }
    for (int k = 0; k < 3; ++k) out[k] = s[k] / M;
}

/* Squared edge length used as the MST weight (Sec. 3.1 weights by Euclidean
 * length; READING: the square, which orders edges identically, evaluated as
 * (dx*dx + dy*dy) + dz*dz with d = x_j - x_i, so w_ij = w_ji bit for bit). */
static double edge_w(const double *xi, const double *xj) {
    double dx = xj[0] - xi[0], dy = xj[1] - xi[1], dz = xj[2] - xi[2];
    return (dx * dx + dy * dy) + dz * dz;
}

/* Strict total order on edges: (w, min(i,j), max(i,j)) lexicographic.  Makes the
 * MST unique (Sec. 3.1: unique weights give a unique MST). */
static int key_less(double w1, int a1, int b1, double w2, int a2, int b2) {
    int lo1 = a1 < b1 ? a1 : b1, hi1 = a1 < b1 ? b1 : a1;
    int lo2 = a2 < b2 ? a2 : b2, hi2 = a2 < b2 ? b2 : a2;
    if (w1 < w2) return 1;
    if (w1 > w2) return 0;
    if (lo1 != lo2) return lo1 < lo2;
    return hi1 < hi2;
}

/* Root choice (Sec. 3.2): the body closest to the centre of mass.  Ties go to
 * the lowest index. */
int orc_root_nearest_com(int n, const double *m, const double *x) {
    double c[3];
    com3(n, m, x, c);
    int best = 0;
    double bw = edge_w(c, x);
    for (int i = 1; i < n; ++i) {
        double w = edge_w(c, x + 3 * i);
        if (w < bw) { bw = w; best = i; }
    }
    return best;
}

/* Prim's algorithm on the complete graph (Sec. 3.2).  Starts at `root`, then
 * repeatedly adds the minimum edge joining the tree to a vertex outside it.
 * parent[] and level[] are assigned as vertices are added, so edges point away
 * from the root and order[] is the order of addition (Sec. 3.4). */
int orc_mst_prim(int n, const double *x, int root, int *parent, int *level, int *order) {
    if (n < 1 || root < 0 || root >= n) return ORC_E_INVAL;
    char *in = (char *)calloc((size_t)n, 1);
    double *bw = (double *)malloc(sizeof(double) * (size_t)n);
    int *bu = (int *)malloc(sizeof(int) * (size_t)n);
    if (!in || !bw || !bu) { free(in); free(bw); free(bu); return ORC_E_NOMEM; }
    in[root] = 1; parent[root] = -1; level[root] = 0; order[0] = root;
    for (int v = 0; v < n; ++v) {
        if (v == root) continue;
        bw[v] = edge_w(x + 3 * root, x + 3 * v);
        bu[v] = root;
    }
    for (int step = 1; step < n; ++step) {
        int pick = -1;
        for (int v = 0; v < n; ++v) {
            if (in[v]) continue;
            if (pick < 0 || key_less(bw[v], bu[v], v, bw[pick], bu[pick], pick)) pick = v;
        }
        in[pick] = 1;
        parent[pick] = bu[pick];
        level[pick] = level[bu[pick]] + 1;
        order[step] = pick;
        for (int u = 0; u < n; ++u) {
            if (in[u]) continue;
            double w = edge_w(x + 3 * pick, x + 3 * u);
            if (key_less(w, pick, u, bw[u], bu[u], u)) { bw[u] = w; bu[u] = pick; }
        }
    }
    free(in); free(bw); free(bu);
    return ORC_OK;
}

/* Levels and a parents-before-children order from a parent array (root has
 * parent -1).  Returns the root, or -1 if parent[] is not a rooted tree. */
int orc_tree_levels(int n, const int *parent, int *level, int *order) {
    int root = -1;
    for (int v = 0; v < n; ++v) {
        if (parent[v] < 0) { if (root >= 0) return -1; root = v; }
        else if (parent[v] >= n || parent[v] == v) return -1;
    }
    if (root < 0) return -1;
    for (int v = 0; v < n; ++v) level[v] = -1;
    level[root] = 0;
    /* walk each vertex up to a vertex of known level (with a cycle guard) */
    for (int v = 0; v < n; ++v) {
        int u = v, len = 0;
        while (level[u] < 0) { u = parent[u]; if (++len > n) return -1; }
        int L = level[u];
        u = v;
        /* assign levels top-down along the walked path */
        int depth = len;
        while (level[u] < 0) { level[u] = L + depth; u = parent[u]; --depth; }
    }
    /* counting sort by level, ties by vertex id */
    int maxL = 0;
    for (int v = 0; v < n; ++v) if (level[v] > maxL) maxL = level[v];
    int *cnt = (int *)calloc((size_t)maxL + 2, sizeof(int));
    if (!cnt) return -1;
    for (int v = 0; v < n; ++v) cnt[level[v] + 1]++;
    for (int l = 0; l <= maxL; ++l) cnt[l + 1] += cnt[l];
    for (int v = 0; v < n; ++v) order[cnt[level[v]]++] = v;
    free(cnt);
    return root;
}

/* ---- Divide-and-conquer spanning tree (Sec. 3.3) ----
 *
 * The bodies are split into about sqrt(N) groups by an octree; each group's
 * minimum spanning tree is found, and so is the minimum spanning tree of the
 * meta-graph whose vertices are the groups and whose edge between two groups
 * weighs as their lightest connecting edge (the cut property makes that edge
 * the one to use).  The union of these edges is a spanning tree, rooted and
 * walked like the exact one.
 *
 * READINGS (the octree is not specified):
 *  - root cell: the axis-aligned cube with lower corner lo = the per-axis
 *    minimum of the positions and side s = the largest per-axis extent; a
 *    body's cell coordinates at the finest depth D = ORC_DC_DEPTH are
 *    (int)((x_c - lo_c) * (2^D / s)), clamped to 2^D - 1 (s = 0: one group);
 *  - a cell holding more than mcap bodies is split into its eight octants
 *    unless it is at depth D; every non-empty unsplit cell is one group.
 *    mcap = ceil(sqrt(N)) gives the ~sqrt(N) groups;
 *  - groups are numbered depth first, octant (bx, by, bz) as 4 bx + 2 by + bz;
 *  - the group trees and the meta-graph tree are the unique minimum spanning
 *    trees under the strict edge order (w, min index, max index).  Pruning
 *    edges by the cycle property before Prim only removes edges that no
 *    minimum spanning tree contains, so it cannot change these trees; it is
 *    left out here.
 */
#define ORC_DC_DEPTH 10

/* Cell coordinates of every body at depth ORC_DC_DEPTH (3 ints per body). */
static void dc_cells(int n, const double *x, int *cc) {
    double lo[3], hi[3];
    for (int c = 0; c < 3; ++c) { lo[c] = x[c]; hi[c] = x[c]; }
    for (int i = 1; i < n; ++i)
        for (int c = 0; c < 3; ++c) {
            if (x[3 * i + c] < lo[c]) lo[c] = x[3 * i + c];
            if (x[3 * i + c] > hi[c]) hi[c] = x[3 * i + c];
        }
    double side = 0.0;
    for (int c = 0; c < 3; ++c) if (hi[c] - lo[c] > side) side = hi[c] - lo[c];
    const int top = (1 << ORC_DC_DEPTH) - 1;
    const double inv = side > 0.0 ? (double)(1 << ORC_DC_DEPTH) / side : 0.0;
    for (int i = 0; i < n; ++i)
        for (int c = 0; c < 3; ++c) {
            int k = (int)((x[3 * i + c] - lo[c]) * inv);
            cc[3 * i + c] = k > top ? top : k;
        }
}

/* Octree split of the bodies in `mem` (ascending indices) at `level`: either
 * one group, or the octants in order. */
static int dc_split(const int *cc, const int *mem, int cnt, int level, int mcap, int *part, int *np) {
    if (cnt <= mcap || level == ORC_DC_DEPTH) {
        for (int k = 0; k < cnt; ++k) part[mem[k]] = *np;
        (*np)++;
        return ORC_OK;
    }
    int *sub = (int *)malloc(sizeof(int) * (size_t)cnt);
    if (!sub) return ORC_E_NOMEM;
    const int bit = ORC_DC_DEPTH - 1 - level;
    int rc = ORC_OK;
    for (int oct = 0; oct < 8 && !rc; ++oct) {
        int m = 0;
        for (int k = 0; k < cnt; ++k) {
            const int *c = cc + 3 * mem[k];
            int o = (((c[0] >> bit) & 1) << 2) | (((c[1] >> bit) & 1) << 1) | ((c[2] >> bit) & 1);
            if (o == oct) sub[m++] = mem[k];
        }
        if (m > 0) rc = dc_split(cc, sub, m, level + 1, mcap, part, np);
    }
    free(sub);
    return rc;
}

/* Prim's algorithm on the complete graph of the bodies mem[0..cnt) (strict
 * order on the global indices); appends the cnt - 1 tree edges to (eu, ev). */
static int dc_prim_group(const double *x, const int *mem, int cnt, int *eu, int *ev, int *ne) {
    if (cnt < 2) return ORC_OK;
    char *in = (char *)calloc((size_t)cnt, 1);
    double *bw = (double *)malloc(sizeof(double) * (size_t)cnt);
    int *bu = (int *)malloc(sizeof(int) * (size_t)cnt);
    if (!in || !bw || !bu) { free(in); free(bw); free(bu); return ORC_E_NOMEM; }
    in[0] = 1;
    for (int k = 1; k < cnt; ++k) { bw[k] = edge_w(x + 3 * mem[0], x + 3 * mem[k]); bu[k] = mem[0]; }
    for (int step = 1; step < cnt; ++step) {
        int pick = -1;
        for (int k = 0; k < cnt; ++k) {
            if (in[k]) continue;
            if (pick < 0 || key_less(bw[k], bu[k], mem[k], bw[pick], bu[pick], mem[pick])) pick = k;
        }
        in[pick] = 1;
        eu[*ne] = bu[pick]; ev[*ne] = mem[pick]; (*ne)++;
        for (int k = 0; k < cnt; ++k) {
            if (in[k]) continue;
            double w = edge_w(x + 3 * mem[pick], x + 3 * mem[k]);
            if (key_less(w, mem[pick], mem[k], bw[k], bu[k], mem[k])) { bw[k] = w; bu[k] = mem[pick]; }
        }
    }
    free(in); free(bw); free(bu);
    return ORC_OK;
}

/* Divide-and-conquer spanning tree rooted at `root` (parents, levels and a
 * parents-first order), with each body's group in part[] and the number of
 * groups in *nparts.  mcap <= 0 means ceil(sqrt(n)). */
int orc_mst_dc(int n, const double *x, int root, int mcap, int *parent, int *level, int *order, int *part,
               int *nparts) {
    if (n < 1 || root < 0 || root >= n) return ORC_E_INVAL;
    if (mcap <= 0) mcap = (int)ceil(sqrt((double)n));
    int *cc = (int *)malloc(sizeof(int) * 3 * (size_t)n), *all = (int *)malloc(sizeof(int) * (size_t)n);
    int *eu = (int *)malloc(sizeof(int) * (size_t)n), *ev = (int *)malloc(sizeof(int) * (size_t)n);
    int *mem = (int *)malloc(sizeof(int) * (size_t)n), *goff = (int *)calloc((size_t)n + 1, sizeof(int));
    char *inT = (char *)calloc((size_t)n, 1);
    double *bw = (double *)malloc(sizeof(double) * (size_t)n);
    int *blo = (int *)malloc(sizeof(int) * (size_t)n), *bhi = (int *)malloc(sizeof(int) * (size_t)n);
    int *adj = (int *)malloc(sizeof(int) * 2 * (size_t)n), *aoff = (int *)calloc((size_t)n + 1, sizeof(int));
    int *queue = (int *)malloc(sizeof(int) * (size_t)n);
    int rc = ORC_OK, np = 0, ne = 0;
    if (!cc || !all || !eu || !ev || !mem || !goff || !inT || !bw || !blo || !bhi || !adj || !aoff || !queue) {
        rc = ORC_E_NOMEM;
        goto out;
    }
    /* 1. octree groups */
    dc_cells(n, x, cc);
    for (int i = 0; i < n; ++i) all[i] = i;
    if ((rc = dc_split(cc, all, n, 0, mcap, part, &np))) goto out;
    *nparts = np;
    /* members of each group, ascending index */
    for (int i = 0; i < n; ++i) goff[part[i] + 1]++;
    for (int g = 0; g < np; ++g) goff[g + 1] += goff[g];
    {
        int *fill = (int *)malloc(sizeof(int) * (size_t)np);
        if (!fill) { rc = ORC_E_NOMEM; goto out; }
        for (int g = 0; g < np; ++g) fill[g] = goff[g];
        for (int i = 0; i < n; ++i) mem[fill[part[i]]++] = i;
        free(fill);
    }
    /* 2. each group's minimum spanning tree */
    for (int g = 0; g < np && !rc; ++g) rc = dc_prim_group(x, mem + goff[g], goff[g + 1] - goff[g], eu, ev, &ne);
    if (rc) goto out;
    /* 3. Prim on the meta-graph: the weight of the meta edge (a, b) is the
     * lightest edge between groups a and b, found when a joins the tree */
    for (int g = 0; g < np; ++g) { bw[g] = INFINITY; blo[g] = -1; bhi[g] = -1; }
    inT[0] = 1;
    for (int added = 0, cur = 0; added < np - 1; ++added) {
        for (int k = goff[cur]; k < goff[cur + 1]; ++k) {
            const int u = mem[k];
            for (int v = 0; v < n; ++v) {
                const int g = part[v];
                if (inT[g]) continue;
                double w = edge_w(x + 3 * u, x + 3 * v);
                int lo = u < v ? u : v, hi = u < v ? v : u;
                if (blo[g] < 0 || key_less(w, lo, hi, bw[g], blo[g], bhi[g])) { bw[g] = w; blo[g] = lo; bhi[g] = hi; }
            }
        }
        int pick = -1;
        for (int g = 0; g < np; ++g) {
            if (inT[g]) continue;
            if (pick < 0 || key_less(bw[g], blo[g], bhi[g], bw[pick], blo[pick], bhi[pick])) pick = g;
        }
        inT[pick] = 1;
        eu[ne] = blo[pick]; ev[ne] = bhi[pick]; ne++;
        cur = pick;
    }
    /* 4. the union, oriented away from the root (breadth first) and walked */
    for (int e = 0; e < ne; ++e) { aoff[eu[e] + 1]++; aoff[ev[e] + 1]++; }
    for (int i = 0; i < n; ++i) aoff[i + 1] += aoff[i];
    {
        int *fill = (int *)malloc(sizeof(int) * (size_t)n);
        if (!fill) { rc = ORC_E_NOMEM; goto out; }
        for (int i = 0; i < n; ++i) fill[i] = aoff[i];
        for (int e = 0; e < ne; ++e) { adj[fill[eu[e]]++] = ev[e]; adj[fill[ev[e]]++] = eu[e]; }
        free(fill);
    }
    for (int i = 0; i < n; ++i) parent[i] = -2;
    parent[root] = -1;
    {
        int head = 0, tail = 0;
        queue[tail++] = root;
        while (head < tail) {
            const int u = queue[head++];
            for (int k = aoff[u]; k < aoff[u + 1]; ++k) {
                const int v = adj[k];
                if (parent[v] != -2) continue;
                parent[v] = u;
                queue[tail++] = v;
            }
        }
        if (tail != n) { rc = ORC_E_INVAL; goto out; }
    }
    if (orc_tree_levels(n, parent, level, order) != root) rc = ORC_E_INVAL;
out:
    free(cc); free(all); free(eu); free(ev); free(mem); free(goff); free(inT); free(bw); free(blo); free(bhi);
    free(adj); free(aoff); free(queue);
    return rc;
}

/* The tree builder of the driver: exact (Sec. 3.2) or divide-and-conquer (Sec. 3.3). */
static int build_tree(int n, const double *x, int root, const orc_params *p, int *parent, int *level,
                      int *order) {
    if (p && p->mst_method == 1) {
        int *part = (int *)malloc(sizeof(int) * (size_t)n), np = 0;
        if (!part) return ORC_E_NOMEM;
        int rc = orc_mst_dc(n, x, root, 0, parent, level, order, part, &np);
        free(part);
        return rc;
    }
    return orc_mst_prim(n, x, root, parent, level, order);
}

/* Deconstruction (Sec. 2.2 / 3.4): original-frame positions relative to the
 * root, rho_root = 0 and rho_v = rho_parent(v) + X_v, parents first. */
void orc_deconstruct(int n, const int *parent, const int *order, const double *X, double *rho) {
    int root = order[0];
    rho[3 * root] = rho[3 * root + 1] = rho[3 * root + 2] = 0.0;
    for (int k = 1; k < n; ++k) {
        int v = order[k], p = parent[v];
        for (int c = 0; c < 3; ++c) rho[3 * v + c] = rho[3 * p + c] + X[3 * v + c];
    }
}

/* Tree closeness by the lowest common ancestor, eq. LCA: i and j are close iff
 * (L(i) - L(LCA)) + (L(j) - L(LCA)) <= N_d.  Climbs at most N_d steps from each
 * side.  On success returns 1 and the two climb lengths a (from i) and b (from j). */
static int tree_close(int i, int j, const int *parent, const int *level, int nd, int *pa, int *pb) {
    int di = level[i] - level[j];
    if (di > nd || -di > nd) return 0;
    int anc[16];
    int u = i;
    int na = 0;
    for (int a = 0; a <= nd; ++a) {
        anc[na++] = u;
        if (parent[u] < 0) break;
        u = parent[u];
    }
    int w = j;
    for (int b = 0; b <= nd; ++b) {
        for (int a = 0; a < na && a + b <= nd; ++a) {
            if (anc[a] == w) { *pa = a; *pb = b; return 1; }
        }
        if (parent[w] < 0) break;
        w = parent[w];
    }
    return 0;
}

/* Sum of the edge vectors on the path from the ancestor `steps` levels above v
 * down to v, accumulated top-down (the vector from that ancestor to v). */
static void path_down(int v, int steps, const int *parent, const double *X, double out[3]) {
    int path[16];
    int u = v;
    for (int s = 0; s < steps; ++s) { path[s] = u; u = parent[u]; }
    out[0] = out[1] = out[2] = 0.0;
    for (int s = steps - 1; s >= 0; --s)
        for (int c = 0; c < 3; ++c) out[c] = out[c] + X[3 * path[s] + c];
}

/* Separation vector d_ij = r_j - r_i (Sec. 3.4 final rule): for pairs within
 * N_d tree edges, the walk i -> LCA -> j summed from MST edge vectors, written
 * as S_j - S_i with S_v the LCA-to-v path sum; otherwise rho_j - rho_i.
 * Returns 1 if the MST path was used.  d_ji = -d_ij bitwise. */
int orc_separation(int i, int j, const int *parent, const int *level, const double *X,
                   const double *rho, int nd, double d[3]) {
    int a, b;
    if (i != j && nd > 0 && tree_close(i, j, parent, level, nd, &a, &b)) {
        double si[3], sj[3];
        path_down(i, a, parent, X, si);
        path_down(j, b, parent, X, sj);
        for (int c = 0; c < 3; ++c) d[c] = sj[c] - si[c];
        return 1;
    }
    for (int c = 0; c < 3; ++c) d[c] = rho[3 * j + c] - rho[3 * i + c];
    return 0;
}

/* Newtonian accelerations and force function (Sec. 2.1):
 *   a_i = G sum_{j!=i} m_j d_ij / |d_ij|^3,  phi_i = sum_{j!=i} m_j / |d_ij|,
 *   U = (G/2) sum_i m_i phi_i.
 * With beta != 0 also Omega = (G/2) sum_i mo_i sum_{j!=i} mo_j/|d_ij| and its
 * gradient dOm_i = G mo_i sum_j mo_j d_ij/|d_ij|^3, where mo_i = m_i if
 * m_i <= omega_mass_max else 0 (READING: Sec. 2.1 gives a force function of
 * the lightest bodies as its example of Omega).  Separations follow
 * orc_separation. */
int orc_force(int n, const double *m, const int *parent, const int *level, const double *X,
              const double *rho, const orc_params *p, double *acc, double *phi,
              double *U, double *Om, double *dOm) {
    const int nd = p->n_d;
    const int want_om = p->beta != 0.0;
    double *mo = NULL, *pom = NULL;
    if (want_om) {
        mo = (double *)malloc(sizeof(double) * (size_t)n);
        pom = (double *)malloc(sizeof(double) * (size_t)n);
        if (!mo || !pom) { free(mo); free(pom); return ORC_E_NOMEM; }
        for (int i = 0; i < n; ++i) mo[i] = (m[i] <= p->omega_mass_max) ? m[i] : 0.0;
    }
#ifdef _OPENMP
    int nt = p->nthreads > 0 ? p->nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 8) num_threads(nt)
#endif
    for (int i = 0; i < n; ++i) {
        double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
        double ox = 0.0, oy = 0.0, oz = 0.0, po = 0.0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double d[3];
            orc_separation(i, j, parent, level, X, rho, nd, d);
            double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
            double rinv = 1.0 / sqrt(r2);
            double rinv3 = (rinv * rinv) * rinv;
            double s = m[j] * rinv3;
            ax = ax + s * d[0];
            ay = ay + s * d[1];
            az = az + s * d[2];
            ph = ph + m[j] * rinv;
            if (want_om) {
                double so = mo[j] * rinv3;
                ox = ox + so * d[0];
                oy = oy + so * d[1];
                oz = oz + so * d[2];
                po = po + mo[j] * rinv;
            }
        }
        acc[3 * i] = p->G * ax;
        acc[3 * i + 1] = p->G * ay;
        acc[3 * i + 2] = p->G * az;
        phi[i] = ph;
        if (want_om) {
            dOm[3 * i] = p->G * mo[i] * ox;
            dOm[3 * i + 1] = p->G * mo[i] * oy;
            dOm[3 * i + 2] = p->G * mo[i] * oz;
            pom[i] = po;
        }
    }
    nsum su;
    ns_init(&su);
    for (int i = 0; i < n; ++i) ns_add(&su, m[i] * phi[i]);
    *U = 0.5 * p->G * ns_get(&su);
    if (want_om) {
        nsum so;
        ns_init(&so);
        for (int i = 0; i < n; ++i) ns_add(&so, mo[i] * pom[i]);
        *Om = 0.5 * p->G * ns_get(&so);
        free(mo); free(pom);
    } else {
        *Om = 0.0;
        if (dOm) memset(dOm, 0, sizeof(double) * 3 * (size_t)n);
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* External perturbation f_i (Sec. 2.1: an acceleration that depends only on
 * the body's position, added to the Newtonian one).  The family offered here:
 * a uniform acceleration g plus np fixed Plummer-softened point masses,
 * pt[k] = (M_k, X_k, Y_k, Z_k, b_k):
 *   f(r) = g + G sum_k M_k (R_k - r) / (|R_k - r|^2 + b_k^2)^(3/2),
 * the gradient field of Phi(r) = -g.r - G sum_k M_k / sqrt(|r - R_k|^2 + b_k^2). */
typedef struct {
    int np;
    double g[3];
    const double *pt;
} orc_ext;

static void ext_accel(const orc_ext *e, double G, const double *r, double *f) {
    for (int c = 0; c < 3; ++c) f[c] = e->g[c];
    for (int k = 0; k < e->np; ++k) {
        const double *q = e->pt + 5 * k;
        double d[3] = {q[1] - r[0], q[2] - r[1], q[3] - r[2]};
        double s2 = ((d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]) + q[4] * q[4];
        double w = G * q[0] / (s2 * sqrt(s2));
        for (int c = 0; c < 3; ++c) f[c] = f[c] + w * d[c];
    }
}

/* f at n positions r[n][3] (exported for the field's own pins). */
int orc_external_accel(int np, const double *g, const double *pt, double G, int n, const double *r, double *f) {
    if (np < 0 || n < 0) return ORC_E_INVAL;
    orc_ext e;
    e.np = np; e.pt = pt;
    for (int c = 0; c < 3; ++c) e.g[c] = g[c];
    for (int i = 0; i < n; ++i) ext_accel(&e, G, r + 3 * i, f + 3 * i);
    return ORC_OK;
}

/* ------------------------------------------------------------------ */
/* The integrated state (READING of Sec. 2.2 with Sec. 3.4): MST edge vectors
 * X_v, V_v (row v = the edge from parent(v) to v; the root row is zero), the
 * centre of mass r_cm, v_cm, physical time t, binding energy B = -H and the TTL
 * variable w.  The tree (parent/level/order) is fixed within a GBS step. */
typedef struct {
    int n;
    const double *m;
    int *parent, *level, *order;
    double *X, *V;
    double t, B, w;
    double rcm[3], vcm[3];
    const orc_ext *ext;   /* external perturbation, or NULL */
} ostate;

/* A substep division works on increments from the step's start state y0
 * (READING: the tableau is formed on Y_k - Y_0, which gives the same
 * extrapolation in exact arithmetic because the Neville weights sum to one,
 * but keeps the rounding of large absolute values such as t out of it).
 * Current values are X = X0 + dX, V = V0 + dV, t = t0 + tau, w = w0 + dw. */
typedef struct {
    const ostate *y0;
    double *dX, *dV;
    double tau, dw, drcm[3];
    double dB, dvcm[3];   /* change of B and v_cm under an external perturbation */
} odiv;

/* Scratch buffers for one leapfrog evaluation. */
typedef struct {
    double *rho, *ups, *acc, *phi, *dom, *vt_old, *vt_new, *Xc, *Vc, *fex;
} oscratch;

static int scratch_alloc(oscratch *s, int n) {
    size_t b = sizeof(double) * 3 * (size_t)n;
    s->rho = (double *)malloc(b); s->ups = (double *)malloc(b); s->acc = (double *)malloc(b);
    s->phi = (double *)malloc(b / 3); s->dom = (double *)malloc(b);
    s->vt_old = (double *)malloc(b); s->vt_new = (double *)malloc(b);
    s->Xc = (double *)malloc(b); s->Vc = (double *)malloc(b); s->fex = (double *)malloc(b);
    return (s->rho && s->ups && s->acc && s->phi && s->dom && s->vt_old && s->vt_new && s->Xc && s->Vc && s->fex)
               ? ORC_OK : ORC_E_NOMEM;
}
static void scratch_free(oscratch *s) {
    free(s->rho); free(s->ups); free(s->acc); free(s->phi); free(s->dom); free(s->vt_old); free(s->vt_new);
    free(s->Xc); free(s->Vc); free(s->fex);
}

/* Centre-of-mass-frame velocities from MST velocity edges V (Sec. 2.2: the
 * velocities are transformed back to the original frame) and the kinetic
 * energy T = 1/2 sum m |v|^2 in the COM frame (READING: B = -H is defined with
 * the internal kinetic energy; the uniform COM motion is carried separately). */
static double com_frame_velocities(const ostate *y, const double *V, double *ups, double *vt) {
    const int n = y->n;
    orc_deconstruct(n, y->parent, y->order, V, ups);
    double ub[3];
    com3(n, y->m, ups, ub);
    nsum T;
    ns_init(&T);
    for (int i = 0; i < n; ++i) {
        for (int c = 0; c < 3; ++c) vt[3 * i + c] = ups[3 * i + c] - ub[c];
        double s2 = (vt[3 * i] * vt[3 * i] + vt[3 * i + 1] * vt[3 * i + 1]) + vt[3 * i + 2] * vt[3 * i + 2];
        ns_add(&T, y->m[i] * s2);
    }
    return 0.5 * ns_get(&T);
}

/* Force evaluation at positions given by edge vectors X: rho from the MST
 * (Sec. 2.2 deconstruction), then orc_force. */
static int eval_force(const ostate *y, const double *X, const orc_params *p, oscratch *s, double *U,
                      double *Om) {
    orc_deconstruct(y->n, y->parent, y->order, X, s->rho);
    return orc_force(y->n, y->m, y->parent, y->level, X, s->rho, p, s->acc, s->phi, U, Om, s->dom);
}

/* External accelerations at the bodies' positions r_i = r_cm + (rho_i - rho_bar)
 * (rho as left in s->rho by eval_force, rcm the current centre of mass) into
 * s->fex; returns sum_i m_i f_i / M in Fm. */
static void external_at(const ostate *y, const double *rcm, const orc_params *p, oscratch *s, double *Fm) {
    const int n = y->n;
    double rb[3];
    com3(n, y->m, s->rho, rb);
    for (int i = 0; i < n; ++i) {
        double r[3];
        for (int c = 0; c < 3; ++c) r[c] = rcm[c] + (s->rho[3 * i + c] - rb[c]);
        ext_accel(y->ext, p->G, r, s->fex + 3 * i);
    }
    com3(n, y->m, s->fex, Fm);
}

static void current_X(const odiv *d, double *Xc) {
    const int n = d->y0->n;
    for (int k = 0; k < 3 * n; ++k) Xc[k] = d->y0->X[k] + d->dX[k];
}
static void current_V(const odiv *d, double *Vc) {
    const int n = d->y0->n;
    for (int k = 0; k < 3 * n; ++k) Vc[k] = d->y0->V[k] + d->dV[k];
}

/* Drift D(ds), Sec. 2.1 and the chained equations of Sec. 2.2:
 * dt = ds / (alpha (T + B) + beta w + gamma);  X += dt V;  r_cm += dt v_cm;
 * t += dt. */
static void drift(odiv *d, const orc_params *p, oscratch *s, double ds) {
    const ostate *y = d->y0;
    const int n = y->n;
    current_V(d, s->Vc);
    double T = com_frame_velocities(y, s->Vc, s->ups, s->vt_old);
    double w = y->w + d->dw;
    double dt = ds / ((p->alpha * (T + (y->B + d->dB)) + p->beta * w) + p->gamma);
    for (int v = 0; v < n; ++v) {
        if (y->parent[v] < 0) continue;
        for (int c = 0; c < 3; ++c) d->dX[3 * v + c] = d->dX[3 * v + c] + dt * s->Vc[3 * v + c];
    }
    for (int c = 0; c < 3; ++c) d->drcm[c] = d->drcm[c] + dt * (y->vcm[c] + d->dvcm[c]);
    d->tau = d->tau + dt;
}

/* Kick K(ds): dt = ds / (alpha U + beta Omega + gamma);  V_v += dt (a_v -
 * a_parent(v)) (the MST analogue of A_k in eq. chained);  with beta != 0 also
 * w += dt sum_i dOmega_i . (v_i_old + v_i_new)/2 (TTL, Mikkola & Aarseth 2002).
 * B is unchanged without external perturbations (Sec. 2.1).  With an external
 * field f (READING of Sec. 2.1 with the COM motion split off): every body
 * takes a_i + f_i, so V_v += dt (a_v + f_v - a_q - f_q) and v_cm += dt F/M
 * (F = sum m_i f_i); f is fixed during the kick, so the COM-frame velocities
 * change linearly in t and the binding-energy equation integrates exactly:
 * B -= dt sum_i m_i f_i . (v_i_old + v_i_new)/2 (COM-frame velocities). */
static int kick(odiv *d, const orc_params *p, oscratch *s, double ds, int64_t *nforce) {
    const ostate *y = d->y0;
    const int n = y->n;
    double U, Om;
    current_X(d, s->Xc);
    int rc = eval_force(y, s->Xc, p, s, &U, &Om);
    if (rc) return rc;
    (*nforce)++;
    double dt = ds / ((p->alpha * U + p->beta * Om) + p->gamma);
    double Fm[3] = {0.0, 0.0, 0.0};
    if (y->ext) {
        double rc_now[3];
        for (int c = 0; c < 3; ++c) rc_now[c] = y->rcm[c] + d->drcm[c];
        external_at(y, rc_now, p, s, Fm);
        for (int k = 0; k < 3 * n; ++k) s->acc[k] = s->acc[k] + s->fex[k];
    }
    if (p->beta != 0.0 || y->ext) {
        current_V(d, s->Vc);
        com_frame_velocities(y, s->Vc, s->ups, s->vt_old);
    }
    for (int v = 0; v < n; ++v) {
        int q = y->parent[v];
        if (q < 0) continue;
        for (int c = 0; c < 3; ++c)
            d->dV[3 * v + c] = d->dV[3 * v + c] + dt * (s->acc[3 * v + c] - s->acc[3 * q + c]);
    }
    if (y->ext) {
        current_V(d, s->Vc);
        com_frame_velocities(y, s->Vc, s->ups, s->vt_new);
        nsum db;
        ns_init(&db);
        for (int i = 0; i < n; ++i)
            for (int c = 0; c < 3; ++c)
                ns_add(&db, y->m[i] * (s->fex[3 * i + c] * (0.5 * (s->vt_old[3 * i + c] + s->vt_new[3 * i + c]))));
        d->dB = d->dB - dt * ns_get(&db);
        for (int c = 0; c < 3; ++c) d->dvcm[c] = d->dvcm[c] + dt * Fm[c];
    }
    if (p->beta != 0.0) {
        current_V(d, s->Vc);
        com_frame_velocities(y, s->Vc, s->ups, s->vt_new);
        nsum dw;
        ns_init(&dw);
        for (int i = 0; i < n; ++i)
            for (int c = 0; c < 3; ++c)
                ns_add(&dw, s->dom[3 * i + c] * (0.5 * (s->vt_old[3 * i + c] + s->vt_new[3 * i + c])));
        d->dw = d->dw + dt * ns_get(&dw);
    }
    return ORC_OK;
}

/* Leapfrog with n substeps over the fictitious interval H (Sec. 2.3):
 * D(H/2n) [K(H/n) D(H/n)]^(n-1) K(H/n) D(H/2n), starting from zero increments. */
static int leapfrog(odiv *d, const orc_params *p, oscratch *s, double H, int nsub, int64_t *nforce) {
    const int n = d->y0->n;
    memset(d->dX, 0, sizeof(double) * 3 * (size_t)n);
    memset(d->dV, 0, sizeof(double) * 3 * (size_t)n);
    d->tau = 0.0; d->dw = 0.0; d->drcm[0] = d->drcm[1] = d->drcm[2] = 0.0;
    d->dB = 0.0; d->dvcm[0] = d->dvcm[1] = d->dvcm[2] = 0.0;
    double h = H / (double)nsub;
    drift(d, p, s, 0.5 * h);
    for (int k = 0; k < nsub - 1; ++k) {
        int rc = kick(d, p, s, h, nforce);
        if (rc) return rc;
        drift(d, p, s, h);
    }
    int rc = kick(d, p, s, h, nforce);
    if (rc) return rc;
    drift(d, p, s, 0.5 * h);
    return ORC_OK;
}

/* Flattened extrapolated variables: X (3n), V (3n), t, r_cm (3), w, B, v_cm (3)
 * (B and v_cm change only under an external perturbation). */
static int nvars(int n) { return 6 * n + 9; }
static void pack_state(const ostate *y, double *out) {
    const int n = y->n;
    memcpy(out, y->X, sizeof(double) * 3 * (size_t)n);
    memcpy(out + 3 * n, y->V, sizeof(double) * 3 * (size_t)n);
    out[6 * n] = y->t;
    out[6 * n + 1] = y->rcm[0]; out[6 * n + 2] = y->rcm[1]; out[6 * n + 3] = y->rcm[2];
    out[6 * n + 4] = y->w;
    out[6 * n + 5] = y->B;
    out[6 * n + 6] = y->vcm[0]; out[6 * n + 7] = y->vcm[1]; out[6 * n + 8] = y->vcm[2];
}
static void pack_incr(const odiv *d, double *out) {
    const int n = d->y0->n;
    memcpy(out, d->dX, sizeof(double) * 3 * (size_t)n);
    memcpy(out + 3 * n, d->dV, sizeof(double) * 3 * (size_t)n);
    out[6 * n] = d->tau;
    out[6 * n + 1] = d->drcm[0]; out[6 * n + 2] = d->drcm[1]; out[6 * n + 3] = d->drcm[2];
    out[6 * n + 4] = d->dw;
    out[6 * n + 5] = d->dB;
    out[6 * n + 6] = d->dvcm[0]; out[6 * n + 7] = d->dvcm[1]; out[6 * n + 8] = d->dvcm[2];
}
/* y += increments */
static void apply_incr(ostate *y, const double *in) {
    const int n = y->n;
    for (int k = 0; k < 3 * n; ++k) { y->X[k] = y->X[k] + in[k]; y->V[k] = y->V[k] + in[3 * n + k]; }
    y->t = y->t + in[6 * n];
    for (int c = 0; c < 3; ++c) y->rcm[c] = y->rcm[c] + in[6 * n + 1 + c];
    y->w = y->w + in[6 * n + 4];
    y->B = y->B + in[6 * n + 5];
    for (int c = 0; c < 3; ++c) y->vcm[c] = y->vcm[c] + in[6 * n + 6 + c];
}

/* Aitken-Neville polynomial extrapolation to h -> 0 in the variable h^2
 * (Sec. 2.3: the leapfrog error has only even powers; Sec. 4.2: Neville-Aitken).
 * tab holds k_fix rows of L values (row k = result of division n_k).
 * On return diag[k] = T_{k,k} for every k (the extrapolation using rows 0..k). */
int orc_neville(int kf, int L, const int *nk, const double *tab, double *diag) {
    /* column j of row k: T_{k,j+1} = T_{k,j} + (T_{k,j} - T_{k-1,j}) / ((n_k/n_{k-j})^2 - 1) */
    double *prev = (double *)malloc(sizeof(double) * (size_t)L * (size_t)kf);
    double *cur = (double *)malloc(sizeof(double) * (size_t)L * (size_t)kf);
    if (!prev || !cur) { free(prev); free(cur); return ORC_E_NOMEM; }
    /* prev = row k-1's entries T_{k-1,0..k-1}; cur = row k */
    for (int v = 0; v < L; ++v) { prev[v] = tab[v]; diag[v] = tab[v]; }
    for (int k = 1; k < kf; ++k) {
        for (int v = 0; v < L; ++v) cur[v] = tab[(size_t)k * L + v];
        for (int j = 1; j <= k; ++j) {
            double r = (double)nk[k] / (double)nk[k - j];
            double den = r * r - 1.0;
            for (int v = 0; v < L; ++v) {
                double a = cur[(size_t)(j - 1) * L + v];
                double b = prev[(size_t)(j - 1) * L + v];
                cur[(size_t)j * L + v] = a + (a - b) / den;
            }
        }
        for (int v = 0; v < L; ++v) diag[(size_t)k * L + v] = cur[(size_t)k * L + v];
        double *tmp = prev; prev = cur; cur = tmp;
    }
    free(prev); free(cur);
    return ORC_OK;
}

/* Euclidean norm of a short vector. */
static double norm_k(const double *a, int k) {
    double s = 0.0;
    for (int c = 0; c < k; ++c) s = s + a[c] * a[c];
    return sqrt(s);
}

/* Error measure of eq. gbs-criterion (READING): for every variable group g
 * (each X_v and each V_v as a 3-vector; t; r_cm; w when beta != 0; B and
 * v_cm under an external perturbation)
 * READING for the centre-of-mass groups r_cm and v_cm: their value can start
 * at the rounding level (a system at rest at the origin), where the linear
 * predictor S + hS' gives no scale; the denominator is then the larger of
 * |S(s0) + hS'(s0)| and |S(s0) + dS_total|, the extrapolated end value.
 *   eps_g = |dS_g| / |S_g(s0) + (H/n) S'_g(s0)|,
 * skipped when the denominator is zero; eps = max_g eps_g.  A non-finite
 * value anywhere gives eps = +inf. */
static double gbs_error(const ostate *y0, const double *dS, const double *S0, const double *dS0ds,
                        const double *inc, double hn, int beta_on) {
    const int n = y0->n;
    double eps = 0.0;
    for (int g = 0; g < 2 * n + 5; ++g) {
        int off, k;
        if (g < 2 * n) {
            int v = g % n;
            if (y0->parent[v] < 0) continue;
            off = 3 * g; k = 3;   /* X rows 0..n-1, V rows n..2n-1 */
        } else if (g == 2 * n) { off = 6 * n; k = 1; }
        else if (g == 2 * n + 1) { off = 6 * n + 1; k = 3; }
        else if (g == 2 * n + 2) { if (!beta_on) continue; off = 6 * n + 4; k = 1; }
        else if (g == 2 * n + 3) { if (!y0->ext) continue; off = 6 * n + 5; k = 1; }
        else { if (!y0->ext) continue; off = 6 * n + 6; k = 3; }
        double num[3], den[3], end[3];
        for (int c = 0; c < k; ++c) {
            num[c] = dS[off + c];
            den[c] = S0[off + c] + hn * dS0ds[off + c];
            end[c] = S0[off + c] + inc[off + c];
            if (!isfinite(num[c])) return INFINITY;
        }
        double dd = norm_k(den, k);
        if (g == 2 * n + 1 || g == 2 * n + 4) {   /* r_cm, v_cm */
            double de = norm_k(end, k);
            if (de > dd) dd = de;
        }
        if (!(dd > 0.0)) continue;
        double e = norm_k(num, k) / dd;
        if (isnan(e)) return INFINITY;
        if (e > eps) eps = e;
    }
    return eps;
}

/* Start-of-step quantities for eq. gbs-criterion: S(s0) and S'(s0) (one force
 * evaluation at the start state, READING) and the force function at the start
 * state, which the driver's end-time clip also uses (Sec. 2.4). */
static int start_eval(ostate *y, const orc_params *p, oscratch *s, double *S0, double *dS0,
                      double *gk_out, int64_t *nforce) {
    const int n = y->n;
    double U0, Om0;
    pack_state(y, S0);
    memset(dS0, 0, sizeof(double) * (size_t)nvars(n));
    int rc = eval_force(y, y->X, p, s, &U0, &Om0);
    if (rc) return rc;
    (*nforce)++;
    double T0 = com_frame_velocities(y, y->V, s->ups, s->vt_old);
    double gd = (p->alpha * (T0 + y->B) + p->beta * y->w) + p->gamma;
    double gk = (p->alpha * U0 + p->beta * Om0) + p->gamma;
    double Fm[3] = {0.0, 0.0, 0.0};
    if (y->ext) {
        external_at(y, y->rcm, p, s, Fm);
        for (int k = 0; k < 3 * n; ++k) s->acc[k] = s->acc[k] + s->fex[k];
        nsum db;
        ns_init(&db);
        for (int i = 0; i < n; ++i)
            for (int c = 0; c < 3; ++c) ns_add(&db, y->m[i] * (s->fex[3 * i + c] * s->vt_old[3 * i + c]));
        dS0[6 * n + 5] = -ns_get(&db) / gk;
        for (int c = 0; c < 3; ++c) dS0[6 * n + 6 + c] = Fm[c] / gk;
    }
    for (int v = 0; v < n; ++v) {
        int q = y->parent[v];
        if (q < 0) continue;
        for (int c = 0; c < 3; ++c) {
            dS0[3 * v + c] = y->V[3 * v + c] / gd;
            dS0[3 * n + 3 * v + c] = (s->acc[3 * v + c] - s->acc[3 * q + c]) / gk;
        }
    }
    dS0[6 * n] = 1.0 / gd;
    for (int c = 0; c < 3; ++c) dS0[6 * n + 1 + c] = y->vcm[c] / gd;
    if (p->beta != 0.0) {
        nsum dw;
        ns_init(&dw);
        for (int i = 0; i < n; ++i)
            for (int c = 0; c < 3; ++c) ns_add(&dw, s->dom[3 * i + c] * s->vt_old[3 * i + c]);
        dS0[6 * n + 4] = ns_get(&dw) / gk;
    }
    *gk_out = gk;
    return ORC_OK;
}

/* One GBS step (Sec. 2.3 and Sec. 4.2): all k_fix divisions n_k = 2k from the
 * same start state, Neville-Aitken extrapolation, error test at k_fix.  On
 * accept the state is replaced by T_{k_fix,k_fix}.  *h_next follows eq. hnext
 * with a_GBS and the clamps [f_min, f_max] (READING); on reject it is H/2. */
static int gbs_divisions(ostate *y, const orc_params *p, oscratch *s, double H, const double *S0,
                         const double *dS0, int *accepted, double *eps_out, double *h_next,
                         int64_t *nforce) {
    const int n = y->n, kf = p->k_fix, L = nvars(n);
    int rc;
    double *tab = (double *)malloc(sizeof(double) * (size_t)L * (size_t)kf);
    double *diag = (double *)malloc(sizeof(double) * (size_t)L * (size_t)kf);
    double *Xw = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *Vw = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    int *nk = (int *)malloc(sizeof(int) * (size_t)kf);
    if (!tab || !diag || !Xw || !Vw || !nk) { rc = ORC_E_NOMEM; goto done; }
    for (int k = 0; k < kf; ++k) nk[k] = 2 * (k + 1);   /* Deuflhard sequence, eq. seq-deuflhard */
    /* the k_fix divisions (independent of each other, Sec. 4.2) */
    for (int k = 0; k < kf; ++k) {
        odiv d;
        d.y0 = y; d.dX = Xw; d.dV = Vw;
        rc = leapfrog(&d, p, s, H, nk[k], nforce);
        if (rc) goto done;
        pack_incr(&d, tab + (size_t)k * L);
    }
    rc = orc_neville(kf, L, nk, tab, diag);
    if (rc) goto done;
    {
        /* dS_k = T_{k,k} - T_{k-1,k-1} (Sec. 4.2); judged at k_fix, or (accept_rule 1,
         * the serial criterion of Sec. 2.3) at the first k whose eps_k <= eta */
        double *dS = tab; /* reuse */
        int k_first = p->accept_rule == 1 ? 2 : kf, kacc = 0;
        double eps = 0.0;
        for (int k = k_first; k <= kf; ++k) {
            for (int v = 0; v < L; ++v) dS[v] = diag[(size_t)(k - 1) * L + v] - diag[(size_t)(k - 2) * L + v];
            eps = gbs_error(y, dS, S0, dS0, diag + (size_t)(k - 1) * L, H / (double)nk[k - 1], p->beta != 0.0);
            if (eps <= p->eta) { kacc = k; break; }
        }
        *eps_out = eps;
        *accepted = kacc > 0;
        if (*accepted) {
            apply_incr(y, diag + (size_t)(kacc - 1) * L);
            double e = eps > 1e-300 ? eps : 1e-300;
            double f = p->a_gbs * pow(p->eta / e, 1.0 / (double)(2 * kacc - 1));
            if (f < p->f_min) f = p->f_min;
            if (f > p->f_max) f = p->f_max;
            *h_next = H * f;
        } else {
            *h_next = 0.5 * H;
        }
    }
    rc = ORC_OK;
done:
    free(tab); free(diag); free(Xw); free(Vw); free(nk);
    return rc;
}

static int gbs_step(ostate *y, const orc_params *p, oscratch *s, double H, int *accepted,
                    double *eps_out, double *h_next, int64_t *nforce) {
    const int L = nvars(y->n);
    double *S0 = (double *)malloc(sizeof(double) * (size_t)L);
    double *dS0 = (double *)malloc(sizeof(double) * (size_t)L);
    double gk;
    int rc = (S0 && dS0) ? ORC_OK : ORC_E_NOMEM;
    if (!rc) rc = start_eval(y, p, s, S0, dS0, &gk, nforce);
    if (!rc) rc = gbs_divisions(y, p, s, H, S0, dS0, accepted, eps_out, h_next, nforce);
    free(S0); free(dS0);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Exported single-stage entry points (state passed as arrays; scal holds
 * t, B, w, r_cm[3], v_cm[3]). */

static int make_state(ostate *y, int n, const double *m, int *parent, int *level, int *order,
                      double *X, double *V, const double *scal) {
    y->n = n; y->m = m; y->parent = parent; y->level = level; y->order = order;
    y->X = X; y->V = V;
    if (orc_tree_levels(n, parent, level, order) < 0) return ORC_E_INVAL;
    y->t = scal[0]; y->B = scal[1]; y->w = scal[2];
    y->ext = NULL;
    for (int c = 0; c < 3; ++c) { y->rcm[c] = scal[3 + c]; y->vcm[c] = scal[6 + c]; }
    return ORC_OK;
}
static void store_scal(const ostate *y, double *scal) {
    scal[0] = y->t; scal[1] = y->B; scal[2] = y->w;
    for (int c = 0; c < 3; ++c) { scal[3 + c] = y->rcm[c]; scal[6 + c] = y->vcm[c]; }
}

/* Force with MST separations given parent[], edge vectors X and rho. */
int orc_force_tree(int n, const double *m, const int *parent, const double *X, const double *rho,
                   const orc_params *p, double *acc, double *phi, double *U, double *Om, double *dOm) {
    int *level = (int *)malloc(sizeof(int) * (size_t)n), *order = (int *)malloc(sizeof(int) * (size_t)n);
    if (!level || !order) { free(level); free(order); return ORC_E_NOMEM; }
    int rc = orc_tree_levels(n, parent, level, order) < 0 ? ORC_E_INVAL : ORC_OK;
    if (!rc) rc = orc_force(n, m, parent, level, X, rho, p, acc, phi, U, Om, dOm);
    free(level); free(order);
    return rc;
}

/* One leapfrog division with nsub substeps over H, in place. */
int orc_leapfrog(int n, const double *m, int *parent, double *X, double *V, double *scal,
                 const orc_params *p, double H, int nsub, int64_t *nforce) {
    int *level = (int *)malloc(sizeof(int) * (size_t)n), *order = (int *)malloc(sizeof(int) * (size_t)n);
    oscratch s;
    int rc = scratch_alloc(&s, n);
    ostate y;
    double *dX = (double *)malloc(sizeof(double) * 3 * (size_t)n), *dV = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *inc = (double *)malloc(sizeof(double) * (size_t)nvars(n));
    if (!rc && (!level || !order || !dX || !dV || !inc)) rc = ORC_E_NOMEM;
    if (!rc) rc = make_state(&y, n, m, parent, level, order, X, V, scal);
    if (!rc) {
        odiv d;
        d.y0 = &y; d.dX = dX; d.dV = dV;
        rc = leapfrog(&d, p, &s, H, nsub, nforce);
        if (!rc) { pack_incr(&d, inc); apply_incr(&y, inc); }
    }
    if (!rc) store_scal(&y, scal);
    free(dX); free(dV); free(inc);
    scratch_free(&s); free(level); free(order);
    return rc;
}

/* One GBS step, in place on accept. */
int orc_gbs_step(int n, const double *m, int *parent, double *X, double *V, double *scal,
                 const orc_params *p, double H, int *accepted, double *eps, double *h_next,
                 int64_t *nforce) {
    int *level = (int *)malloc(sizeof(int) * (size_t)n), *order = (int *)malloc(sizeof(int) * (size_t)n);
    oscratch s;
    int rc = scratch_alloc(&s, n);
    ostate y;
    if (!rc && (!level || !order)) rc = ORC_E_NOMEM;
    if (!rc) rc = make_state(&y, n, m, parent, level, order, X, V, scal);
    if (!rc) rc = gbs_step(&y, p, &s, H, accepted, eps, h_next, nforce);
    if (!rc) store_scal(&y, scal);
    scratch_free(&s); free(level); free(order);
    return rc;
}

/* Neville extrapolation exported for tests: tab[kf][L] -> diag[kf][L]. */
int orc_neville_export(int kf, int L, const double *tab, double *diag) {
    int nk[64];
    if (kf < 1 || kf > 64) return ORC_E_INVAL;
    for (int k = 0; k < kf; ++k) nk[k] = 2 * (k + 1);
    return orc_neville(kf, L, nk, tab, diag);
}

/* Build the MST state from Cartesian x, v (Sec. 3.2, 3.4): root nearest the
 * COM, Prim tree, edge vectors X_v = x_v - x_parent, V_v likewise. */
static int build_state_p(int n, const double *m, const double *x, const double *v, const orc_params *p,
                         int *parent, double *X, double *V, double *scal);

int orc_build_state(int n, const double *m, const double *x, const double *v,
                    int *parent, double *X, double *V, double *scal) {
    return build_state_p(n, m, x, v, NULL, parent, X, V, scal);
}

/* orc_build_state with the tree builder of params p (NULL: exact). */
static int build_state_p(int n, const double *m, const double *x, const double *v, const orc_params *p,
                         int *parent, double *X, double *V, double *scal) {
    int *level = (int *)malloc(sizeof(int) * (size_t)n), *order = (int *)malloc(sizeof(int) * (size_t)n);
    if (!level || !order) { free(level); free(order); return ORC_E_NOMEM; }
    int root = orc_root_nearest_com(n, m, x);
    int rc = build_tree(n, x, root, p, parent, level, order);
    if (!rc) {
        for (int c = 0; c < 3; ++c) { X[3 * root + c] = 0.0; V[3 * root + c] = 0.0; }
        for (int u = 0; u < n; ++u) {
            int q = parent[u];
            if (q < 0) continue;
            for (int c = 0; c < 3; ++c) {
                X[3 * u + c] = x[3 * u + c] - x[3 * q + c];
                V[3 * u + c] = v[3 * u + c] - v[3 * q + c];
            }
        }
        double rc3[3], vc3[3];
        com3(n, m, x, rc3);
        com3(n, m, v, vc3);
        scal[0] = 0.0; scal[1] = 0.0; scal[2] = 0.0;
        for (int c = 0; c < 3; ++c) { scal[3 + c] = rc3[c]; scal[6 + c] = vc3[c]; }
    }
    free(level); free(order);
    return rc;
}

/* Cartesian positions and velocities from the MST state (Sec. 2.2 deconstruction):
 * x_i = r_cm + (rho_i - rho_bar), v_i = v_cm + (ups_i - ups_bar). */
int orc_state_to_cartesian(int n, const double *m, const int *parent, const double *X, const double *V,
                           const double *scal, double *x, double *v) {
    int *level = (int *)malloc(sizeof(int) * (size_t)n), *order = (int *)malloc(sizeof(int) * (size_t)n);
    double *rho = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    if (!level || !order || !rho) { free(level); free(order); free(rho); return ORC_E_NOMEM; }
    int rc = orc_tree_levels(n, parent, level, order) < 0 ? ORC_E_INVAL : ORC_OK;
    if (!rc) {
        double c[3];
        orc_deconstruct(n, parent, order, X, rho);
        com3(n, m, rho, c);
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < 3; ++k) x[3 * i + k] = scal[3 + k] + (rho[3 * i + k] - c[k]);
        orc_deconstruct(n, parent, order, V, rho);
        com3(n, m, rho, c);
        for (int i = 0; i < n; ++i)
            for (int k = 0; k < 3; ++k) v[3 * i + k] = scal[6 + k] + (rho[3 * i + k] - c[k]);
    }
    free(level); free(order); free(rho);
    return rc;
}

/* MST rebuild during integration (Sec. 3.5: the structure is built,
 * deconstructed and rebuilt).  New tree from rho (root nearest the COM of rho);
 * READING: the edge vector of each new tree edge (q -> u) is the separation the
 * old tree gives for that pair under the close-pair rule (so edges that persist
 * keep their bits, a reversed edge is negated exactly, and only genuinely new
 * far pairs fall back to rho_u - rho_q).  Velocities likewise.  Returns 1 if the
 * parent array changed. */
static int rebuild(ostate *y, const orc_params *p, oscratch *s, int *topo_changed) {
    const int n = y->n;
    int *np = (int *)malloc(sizeof(int) * (size_t)n), *nl = (int *)malloc(sizeof(int) * (size_t)n);
    int *no = (int *)malloc(sizeof(int) * (size_t)n);
    double *nX = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *nV = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    if (!np || !nl || !no || !nX || !nV) { free(np); free(nl); free(no); free(nX); free(nV); return ORC_E_NOMEM; }
    orc_deconstruct(n, y->parent, y->order, y->X, s->rho);
    orc_deconstruct(n, y->parent, y->order, y->V, s->ups);
    int root = orc_root_nearest_com(n, y->m, s->rho);
    int rc = build_tree(n, s->rho, root, p, np, nl, no);
    if (rc) goto out;
    int changed = 0;
    for (int u = 0; u < n; ++u) if (np[u] != y->parent[u]) { changed = 1; break; }
    *topo_changed = changed;
    if (changed) {
        for (int u = 0; u < n; ++u) {
            int q = np[u];
            if (q < 0) { for (int c = 0; c < 3; ++c) { nX[3 * u + c] = 0.0; nV[3 * u + c] = 0.0; } continue; }
            orc_separation(q, u, y->parent, y->level, y->X, s->rho, p->n_d, nX + 3 * u);
            orc_separation(q, u, y->parent, y->level, y->V, s->ups, p->n_d, nV + 3 * u);
        }
        memcpy(y->parent, np, sizeof(int) * (size_t)n);
        memcpy(y->level, nl, sizeof(int) * (size_t)n);
        memcpy(y->order, no, sizeof(int) * (size_t)n);
        memcpy(y->X, nX, sizeof(double) * 3 * (size_t)n);
        memcpy(y->V, nV, sizeof(double) * 3 * (size_t)n);
    }
out:
    free(np); free(nl); free(no); free(nX); free(nV);
    return rc;
}

/* The driver's rebuild (Sec. 3.5) applied to a given state, exported for the
 * tests of the new-edge rule: parent, X and V (edge rows) are replaced by the
 * new tree's and *changed tells whether the tree changed. */
int orc_rebuild_state(int n, const double *m, int *parent, double *X, double *V, const double *scal,
                      const orc_params *p, int *changed) {
    int *level = (int *)malloc(sizeof(int) * (size_t)n), *order = (int *)malloc(sizeof(int) * (size_t)n);
    oscratch s;
    int rc = scratch_alloc(&s, n);
    if (!rc && (!level || !order)) rc = ORC_E_NOMEM;
    ostate y;
    if (!rc) rc = make_state(&y, n, m, parent, level, order, X, V, scal);
    if (!rc) rc = rebuild(&y, p, &s, changed);
    scratch_free(&s);
    free(level); free(order);
    return rc;
}

static int all_finite(int k, const double *a) {
    for (int i = 0; i < k; ++i) if (!isfinite(a[i])) return 0;
    return 1;
}

/* The driver (Sec. 2.4): integrate from t0 to t_end in physical time.
 * First step ds = q U dt (eq. t-aika times a safety factor).  Before each step
 * the predicted end time tau + ds/(alpha U + beta Omega + gamma) is compared
 * with t_end and the step is clipped to land on it; an overshoot is undone with
 * a step of negative ds (the leapfrog is time symmetric), until
 * |t_end - tau| <= t_tol |t_end - t0| or max_time_iter extra steps were taken.
 * Unconverged GBS steps are halved (Sec. 2.3).  x, v are replaced by the state
 * at t_reached. */
static int integrate_impl(int n, const double *m, double *x, double *v, double t0, double t_end,
                          const orc_params *p, orc_stats *st, int64_t max_acc, double *rec_H,
                          int32_t *rec_par, int64_t *n_rec, const orc_ext *ext);

int orc_integrate(int n, const double *m, double *x, double *v, double t0, double t_end,
                  const orc_params *p, orc_stats *st) {
    return integrate_impl(n, m, x, v, t0, t_end, p, st, -1, NULL, NULL, NULL, NULL);
}

/* The driver under the external perturbation of ext_accel (Sec. 2.1):
 * g[3] and np points pt[np][5] = (M, X, Y, Z, b).  Only with beta = 0. */
int orc_integrate_ext(int n, const double *m, double *x, double *v, double t0, double t_end,
                      const orc_params *p, int np, const double *g, const double *pt, orc_stats *st) {
    if (np < 0 || (np > 0 && !pt) || !g || p->beta != 0.0) return ORC_E_INVAL;
    orc_ext e;
    e.np = np; e.pt = pt;
    for (int c = 0; c < 3; ++c) e.g[c] = g[c];
    return integrate_impl(n, m, x, v, t0, t_end, p, st, -1, NULL, NULL, NULL, &e);
}

/* The driver with a record of its accepted steps, for the frozen-controller
 * replay below: for accepted step k < max_acc, rec_H[k] is its fictitious
 * step and rec_par[k*n ..] the MST parent array it used.  Stops after max_acc
 * accepted steps (returning ORC_OK) if t_end is not reached first. */
int orc_integrate_rec(int n, const double *m, double *x, double *v, double t0, double t_end,
                      const orc_params *p, orc_stats *st, int64_t max_acc, double *rec_H,
                      int32_t *rec_par, int64_t *n_rec) {
    if (max_acc < 1 || !rec_H || !rec_par || !n_rec) return ORC_E_INVAL;
    return integrate_impl(n, m, x, v, t0, t_end, p, st, max_acc, rec_H, rec_par, n_rec, NULL);
}

static int integrate_impl(int n, const double *m, double *x, double *v, double t0, double t_end,
                          const orc_params *p, orc_stats *st, int64_t max_acc, double *rec_H,
                          int32_t *rec_par, int64_t *n_rec, const orc_ext *ext) {
    memset(st, 0, sizeof(*st));
    if (n_rec) *n_rec = 0;
    st->t_reached = t0;
    if (n < 2 || p->k_fix < 2 || p->k_fix > 32 || p->n_d < 0 || p->n_d > 8 || !(p->eta > 0.0) ||
        !(p->G > 0.0) || !(t_end != t0) || !isfinite(t0) || !isfinite(t_end))
        return ORC_E_INVAL;
    for (int i = 0; i < n; ++i) if (!(m[i] > 0.0) || !isfinite(m[i])) return ORC_E_INVAL;
    if (!all_finite(3 * n, x) || !all_finite(3 * n, v)) return ORC_E_NONFINITE;
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j)
            if (edge_w(x + 3 * i, x + 3 * j) == 0.0) return ORC_E_COINCIDENT;

    int *parent = (int *)malloc(sizeof(int) * (size_t)n), *level = (int *)malloc(sizeof(int) * (size_t)n);
    int *order = (int *)malloc(sizeof(int) * (size_t)n);
    double *X = (double *)malloc(sizeof(double) * 3 * (size_t)n), *V = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double scal[9];
    oscratch s;
    int rc = scratch_alloc(&s, n);
    if (!rc && (!parent || !level || !order || !X || !V)) rc = ORC_E_NOMEM;
    if (rc) goto out;
    rc = build_state_p(n, m, x, v, p, parent, X, V, scal);
    if (rc) goto out;
    ostate y;
    make_state(&y, n, m, parent, level, order, X, V, scal);
    y.t = t0;
    y.ext = ext;
    {
        double U0, Om0;
        rc = eval_force(&y, y.X, p, &s, &U0, &Om0);
        if (rc) goto out;
        st->force_evals++;
        double T0 = com_frame_velocities(&y, y.V, s.ups, s.vt_old);
        y.B = U0 - T0;                 /* B = -H = -(T - U) */
        y.w = Om0;
        double gk = (p->alpha * U0 + p->beta * Om0) + p->gamma;
        double H = p->h_init > 0.0 ? p->h_init : p->q_first * gk * (t_end - t0);
        const double span = fabs(t_end - t0);
        const int L = nvars(n);
        double *S0 = (double *)malloc(sizeof(double) * (size_t)L);
        double *dS0 = (double *)malloc(sizeof(double) * (size_t)L);
        int halvings = 0, since_rebuild = 0, fresh = 1;
        int64_t iters = 0;
        if (!S0 || !dS0) rc = ORC_E_NOMEM;
        while (!rc) {
            if (st->steps_accepted + st->steps_rejected >= p->max_steps) { rc = ORC_E_MAXSTEPS; break; }
            if (fresh) {
                if (since_rebuild >= p->rebuild_every) {
                    int ch = 0;
                    rc = rebuild(&y, p, &s, &ch);
                    if (rc) break;
                    st->mst_rebuilds++;
                    st->topo_changes += ch;
                    since_rebuild = 0;
                }
                rc = start_eval(&y, p, &s, S0, dS0, &gk, &st->force_evals);
                if (rc) break;
                fresh = 0;
            }
            /* end-time clip with the force function at the step start (Sec. 2.4) */
            double rem = t_end - y.t;
            double dt_est = H / gk;
            int clipped = 0;
            if (dt_est / rem > 1.0 || dt_est / rem < 0.0) { H = gk * rem; clipped = 1; }
            int acc = 0;
            double eps = 0.0, hn = 0.0;
            rc = gbs_divisions(&y, p, &s, H, S0, dS0, &acc, &eps, &hn, &st->force_evals);
            if (rc) break;
            st->eps_last = eps;
            if (!acc) {
                st->steps_rejected++;
                if (++halvings > p->max_halvings) { rc = ORC_E_NOCONV; break; }
                H = hn;
                continue;
            }
            if (rec_H && *n_rec < max_acc) {
                rec_H[*n_rec] = H;
                memcpy(rec_par + (size_t)(*n_rec) * (size_t)n, y.parent, sizeof(int32_t) * (size_t)n);
                ++*n_rec;
            }
            st->steps_accepted++;
            st->h_last = H;
            halvings = 0;
            since_rebuild++;
            fresh = 1;
            if (clipped) iters++;
            H = hn;
            st->h_next = hn;
            if (fabs(t_end - y.t) <= p->t_tol * span) { rc = ORC_OK; break; }
            if (iters > p->max_time_iter) { rc = ORC_W_TIME_TOL; break; }
            if (max_acc > 0 && st->steps_accepted >= max_acc) { rc = ORC_OK; break; }
        }
        free(S0); free(dS0);
        st->time_iters = iters;
    }
    st->t_reached = y.t;
    if (rc == ORC_OK || rc == ORC_W_TIME_TOL || rc == ORC_E_NOCONV || rc == ORC_E_MAXSTEPS) {
        store_scal(&y, scal);
        orc_state_to_cartesian(n, m, parent, X, V, scal, x, v);
    }
out:
    scratch_free(&s);
    free(parent); free(level); free(order); free(X); free(V);
    return rc;
}

/* Plain Cartesian diagnostics (Sec. 5.1): E = T - U, total momentum P and
 * angular momentum L = sum m r x v, Neumaier sums in index order. */
void orc_diagnostics(int n, const double *m, const double *x, const double *v, double G, double *out) {
    nsum T, U, P[3], L[3];
    ns_init(&T); ns_init(&U);
    for (int c = 0; c < 3; ++c) { ns_init(&P[c]); ns_init(&L[c]); }
    for (int i = 0; i < n; ++i) {
        const double *xi = x + 3 * i, *vi = v + 3 * i;
        ns_add(&T, 0.5 * m[i] * ((vi[0] * vi[0] + vi[1] * vi[1]) + vi[2] * vi[2]));
        for (int c = 0; c < 3; ++c) ns_add(&P[c], m[i] * vi[c]);
        ns_add(&L[0], m[i] * (xi[1] * vi[2] - xi[2] * vi[1]));
        ns_add(&L[1], m[i] * (xi[2] * vi[0] - xi[0] * vi[2]));
        ns_add(&L[2], m[i] * (xi[0] * vi[1] - xi[1] * vi[0]));
        for (int j = i + 1; j < n; ++j) ns_add(&U, G * m[i] * m[j] / sqrt(edge_w(xi, x + 3 * j)));
    }
    out[0] = ns_get(&T) - ns_get(&U);
    out[1] = ns_get(&T);
    out[2] = ns_get(&U);
    for (int c = 0; c < 3; ++c) { out[3 + c] = ns_get(&P[c]); out[6 + c] = ns_get(&L[c]); }
}

/* Greedy assignment of substep divisions to groups (Sec. 4.2): largest n_k first
 * to the least-loaded group, ties to the lowest group index.  Returns
 * S_div = sum n_k / max_i C_i (eq. speedup-div); group[k] receives the group
 * of division k. */
double orc_sdiv(int kf, int ndiv, int *group) {
    int64_t C[64] = {0};
    int64_t total = 0;
    if (ndiv < 1 || ndiv > 64) return 0.0;
    for (int k = kf; k >= 1; --k) {
        int nkk = 2 * k;
        int g = 0;
        for (int q = 1; q < ndiv; ++q) if (C[q] < C[g]) g = q;
        C[g] += nkk;
        total += nkk;
        if (group) group[k - 1] = g;
    }
    int64_t mx = 0;
    for (int q = 0; q < ndiv; ++q) if (C[q] > mx) mx = C[q];
    return (double)total / (double)mx;
}

/* ------------------------------------------------------------------ */
/* Frozen-controller replay and its tangent-linear model (the reference for
 * the adjoint; not in the paper).  With the accepted steps H_k and the MST
 * topologies recorded, the integrator is a smooth map from the initial
 * positions and velocities to the end state: discretise, then differentiate. */

/* Rebuild onto a given parent array (Sec. 3.5 with the topology fixed): the
 * edge vector of each new edge is the old tree's separation of that pair
 * under the close-pair rule, as in rebuild(). */
static int rebuild_to(ostate *y, const orc_params *p, oscratch *s, const int32_t *np) {
    const int n = y->n;
    int changed = 0;
    for (int u = 0; u < n; ++u) if (np[u] != y->parent[u]) { changed = 1; break; }
    if (!changed) return ORC_OK;
    int *nl = (int *)malloc(sizeof(int) * (size_t)n), *no = (int *)malloc(sizeof(int) * (size_t)n);
    double *nX = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *nV = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    int rc = ORC_OK;
    if (!nl || !no || !nX || !nV) { rc = ORC_E_NOMEM; goto out; }
    if (orc_tree_levels(n, np, nl, no) < 0) { rc = ORC_E_INVAL; goto out; }
    orc_deconstruct(n, y->parent, y->order, y->X, s->rho);
    orc_deconstruct(n, y->parent, y->order, y->V, s->ups);
    for (int u = 0; u < n; ++u) {
        int q = np[u];
        if (q < 0) { for (int c = 0; c < 3; ++c) { nX[3 * u + c] = 0.0; nV[3 * u + c] = 0.0; } continue; }
        orc_separation(q, u, y->parent, y->level, y->X, s->rho, p->n_d, nX + 3 * u);
        orc_separation(q, u, y->parent, y->level, y->V, s->ups, p->n_d, nV + 3 * u);
    }
    memcpy(y->parent, np, sizeof(int) * (size_t)n);
    memcpy(y->level, nl, sizeof(int) * (size_t)n);
    memcpy(y->order, no, sizeof(int) * (size_t)n);
    memcpy(y->X, nX, sizeof(double) * 3 * (size_t)n);
    memcpy(y->V, nV, sizeof(double) * 3 * (size_t)n);
out:
    free(nl); free(no); free(nX); free(nV);
    return rc;
}

/* One GBS step of fixed length H without the error test (Sec. 2.3): the k_fix
 * divisions, Neville-Aitken, state += T_{k_fix,k_fix} -- the arithmetic of an
 * accepted gbs_divisions(). */
static int replay_step(ostate *y, const orc_params *p, oscratch *s, double H, int64_t *nforce) {
    const int n = y->n, kf = p->k_fix, L = nvars(n);
    int rc = ORC_OK;
    double *tab = (double *)malloc(sizeof(double) * (size_t)L * (size_t)kf);
    double *diag = (double *)malloc(sizeof(double) * (size_t)L * (size_t)kf);
    double *Xw = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *Vw = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    int *nk = (int *)malloc(sizeof(int) * (size_t)kf);
    if (!tab || !diag || !Xw || !Vw || !nk) { rc = ORC_E_NOMEM; goto out; }
    for (int k = 0; k < kf; ++k) nk[k] = 2 * (k + 1);
    for (int k = 0; k < kf && !rc; ++k) {
        odiv d;
        d.y0 = y; d.dX = Xw; d.dV = Vw;
        rc = leapfrog(&d, p, s, H, nk[k], nforce);
        if (!rc) pack_incr(&d, tab + (size_t)k * L);
    }
    if (!rc) rc = orc_neville(kf, L, nk, tab, diag);
    if (!rc) apply_incr(y, diag + (size_t)(kf - 1) * L);
out:
    free(tab); free(diag); free(Xw); free(Vw); free(nk);
    return rc;
}

/* Replay: initial MST state on parents[0], then for k < nsteps a rebuild onto
 * parents[k] (k > 0) and a GBS step of length H[k]; x, v are replaced by the
 * end state and *t_out is its time.  With the record of orc_integrate_rec
 * this repeats that integration bit for bit.  With parents NULL the trees are
 * the driver's own: the MST of x rooted nearest the centre of mass at the
 * start, and the rebuild of Sec. 3.5 before every rebuild_every-th step
 * after it -- the integration of orc_integrate with its accepted step
 * lengths given instead of chosen.  t_steps (nullable, nsteps values)
 * receives the time after each step. */
int orc_replay(int n, const double *m, double *x, double *v, double t0, int64_t nsteps, const double *H,
               const int32_t *parents, const orc_params *p, double *t_out, double *t_steps) {
    if (n < 2 || nsteps < 0 || !H || p->beta != 0.0) return ORC_E_INVAL;
    int *parent = (int *)malloc(sizeof(int) * (size_t)n), *level = (int *)malloc(sizeof(int) * (size_t)n);
    int *order = (int *)malloc(sizeof(int) * (size_t)n);
    double *X = (double *)malloc(sizeof(double) * 3 * (size_t)n), *V = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double scal[9];
    oscratch s;
    int rc = scratch_alloc(&s, n);
    if (!rc && (!parent || !level || !order || !X || !V)) rc = ORC_E_NOMEM;
    if (rc) goto out;
    if (parents) memcpy(parent, parents, sizeof(int) * (size_t)n);
    else if ((rc = build_tree(n, x, orc_root_nearest_com(n, m, x), p, parent, level, order))) goto out;
    if (orc_tree_levels(n, parent, level, order) < 0) { rc = ORC_E_INVAL; goto out; }
    for (int u = 0; u < n; ++u) {
        int q = parent[u];
        for (int c = 0; c < 3; ++c) {
            X[3 * u + c] = q < 0 ? 0.0 : x[3 * u + c] - x[3 * q + c];
            V[3 * u + c] = q < 0 ? 0.0 : v[3 * u + c] - v[3 * q + c];
        }
    }
    {
        double rc3[3], vc3[3];
        com3(n, m, x, rc3);
        com3(n, m, v, vc3);
        scal[0] = t0; scal[1] = 0.0; scal[2] = 0.0;
        for (int c = 0; c < 3; ++c) { scal[3 + c] = rc3[c]; scal[6 + c] = vc3[c]; }
    }
    ostate y;
    make_state(&y, n, m, parent, level, order, X, V, scal);
    {
        double U0, Om0;
        int64_t nf = 0;
        rc = eval_force(&y, y.X, p, &s, &U0, &Om0);
        if (rc) goto out;
        double T0 = com_frame_velocities(&y, y.V, s.ups, s.vt_old);
        y.B = U0 - T0;
        int since_rebuild = 0, ch = 0;
        for (int64_t k = 0; k < nsteps && !rc; ++k) {
            if (parents) {
                if (k > 0) rc = rebuild_to(&y, p, &s, parents + (size_t)k * (size_t)n);
            } else if (since_rebuild >= p->rebuild_every) {
                rc = rebuild(&y, p, &s, &ch);
                since_rebuild = 0;
            }
            if (!rc) rc = replay_step(&y, p, &s, H[k], &nf);
            if (!rc && t_steps) t_steps[k] = y.t;
            since_rebuild++;
        }
    }
    if (!rc) {
        store_scal(&y, scal);
        orc_state_to_cartesian(n, m, parent, X, V, scal, x, v);
        if (t_out) *t_out = y.t;
    }
out:
    scratch_free(&s);
    free(parent); free(level); free(order); free(X); free(V);
    return rc;
}

/* Tangent of the Newtonian force (Sec. 2.1) in Cartesian coordinates r [n][3]:
 * a_i = G sum_j m_j d_ij/|d_ij|^3 with d_ij = r_j - r_i, U = G sum_{i<j} m_i m_j/|d_ij|,
 * and for each of nd directions dr [nd][n][3]:
 *   da_i = G sum_j m_j (I/r^3 - 3 d d^T/r^5)(dr_j - dr_i),  dU = sum_i m_i a_i . dr_i
 * (the derivative of d/|d|^3 and of 1/|d|).  OpenMP over i only.  a, U, da,
 * dU may be NULL. */
int orc_force_tlm(int n, const double *m, const double *r, double G, int nd, const double *dr,
                  double *a, double *U, double *da, double *dU, int nthreads) {
    double *acc = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    double *phi = (double *)malloc(sizeof(double) * (size_t)n);
    if (!acc || !phi) { free(acc); free(phi); return ORC_E_NOMEM; }
#ifdef _OPENMP
    int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nt)
#endif
    for (int i = 0; i < n; ++i) {
        double ax = 0.0, ay = 0.0, az = 0.0, ph = 0.0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            double d0 = r[3 * j] - r[3 * i], d1 = r[3 * j + 1] - r[3 * i + 1], d2 = r[3 * j + 2] - r[3 * i + 2];
            double r2 = (d0 * d0 + d1 * d1) + d2 * d2;
            double ri = 1.0 / sqrt(r2);
            double s3 = m[j] * ((ri * ri) * ri);
            ax = ax + s3 * d0; ay = ay + s3 * d1; az = az + s3 * d2;
            ph = ph + m[j] * ri;
        }
        acc[3 * i] = G * ax; acc[3 * i + 1] = G * ay; acc[3 * i + 2] = G * az;
        phi[i] = ph;
    }
    if (a) memcpy(a, acc, sizeof(double) * 3 * (size_t)n);
    if (U) {
        nsum su;
        ns_init(&su);
        for (int i = 0; i < n; ++i) ns_add(&su, m[i] * phi[i]);
        *U = 0.5 * G * ns_get(&su);
    }
    for (int q = 0; q < nd && da; ++q) {
        const double *t = dr + (size_t)q * 3 * (size_t)n;
        double *o = da + (size_t)q * 3 * (size_t)n;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(nt)
#endif
        for (int i = 0; i < n; ++i) {
            double gx = 0.0, gy = 0.0, gz = 0.0;
            for (int j = 0; j < n; ++j) {
                if (j == i) continue;
                double d0 = r[3 * j] - r[3 * i], d1 = r[3 * j + 1] - r[3 * i + 1], d2 = r[3 * j + 2] - r[3 * i + 2];
                double r2 = (d0 * d0 + d1 * d1) + d2 * d2;
                double ri = 1.0 / sqrt(r2);
                double r3 = (ri * ri) * ri, r5 = r3 * (ri * ri);
                double e0 = t[3 * j] - t[3 * i], e1 = t[3 * j + 1] - t[3 * i + 1], e2 = t[3 * j + 2] - t[3 * i + 2];
                double de = (d0 * e0 + d1 * e1) + d2 * e2;
                gx = gx + m[j] * (e0 * r3 - 3.0 * d0 * de * r5);
                gy = gy + m[j] * (e1 * r3 - 3.0 * d1 * de * r5);
                gz = gz + m[j] * (e2 * r3 - 3.0 * d2 * de * r5);
            }
            o[3 * i] = G * gx; o[3 * i + 1] = G * gy; o[3 * i + 2] = G * gz;
        }
        if (dU) {
            nsum du;
            ns_init(&du);
            for (int i = 0; i < n; ++i)
                for (int c = 0; c < 3; ++c) ns_add(&du, m[i] * (acc[3 * i + c] * t[3 * i + c]));
            dU[q] = ns_get(&du);
        }
    }
    free(acc); free(phi);
    return ORC_OK;
}

/* The frozen-controller map in exact arithmetic does not depend on the
 * coordinates it is evaluated in: the MST transforms and rebuilds are linear
 * changes of variables (Sec. 2.2, 3.5), a drift moves every body by dt v_i
 * and a kick changes every velocity by dt a_i (the MST form is the same
 * update on edge differences; sum_i m_i a_i = 0).  The tangent-linear model
 * is therefore written in Cartesian coordinates: state (r, v, t), constant
 * B = U(r0) - T(v0) (Sec. 2.1, B = -H), and nd tangent directions carried
 * along with it. */
typedef struct {
    int n, nd, nthreads;
    const double *m;
    double G, alpha, gamma, B, t;
    double *r, *v;          /* [n][3] */
    double *dr, *dv;        /* [nd][n][3] */
    double *dt, *dB;        /* [nd] */
} tstate;

typedef struct { double *vc, *a, *da, *dU; } tscratch;

/* T = 1/2 sum m |v - v_cm|^2 and the COM-frame velocities (as com_frame_velocities). */
static double t_kinetic(const tstate *z, double *vc) {
    double vb[3];
    com3(z->n, z->m, z->v, vb);
    nsum T;
    ns_init(&T);
    for (int i = 0; i < z->n; ++i) {
        for (int c = 0; c < 3; ++c) vc[3 * i + c] = z->v[3 * i + c] - vb[c];
        ns_add(&T, z->m[i] * ((vc[3 * i] * vc[3 * i] + vc[3 * i + 1] * vc[3 * i + 1]) + vc[3 * i + 2] * vc[3 * i + 2]));
    }
    return 0.5 * ns_get(&T);
}

/* Drift D(ds): dt = ds/(alpha (T + B) + gamma); r += dt v; t += dt.
 * Tangent: dT = sum m vc . dv; d(dt) = -(dt/g) alpha (dT + dB). */
static void t_drift(tstate *z, tscratch *w, double ds) {
    const int n = z->n;
    double T = t_kinetic(z, w->vc);
    double g = z->alpha * (T + z->B) + z->gamma;
    double dt = ds / g;
    for (int q = 0; q < z->nd; ++q) {
        double *dr = z->dr + (size_t)q * 3 * n, *dv = z->dv + (size_t)q * 3 * n;
        nsum s;
        ns_init(&s);
        for (int i = 0; i < n; ++i)
            for (int c = 0; c < 3; ++c) ns_add(&s, z->m[i] * (w->vc[3 * i + c] * dv[3 * i + c]));
        double ddt = -(dt / g) * (z->alpha * (ns_get(&s) + z->dB[q]));
        for (int k = 0; k < 3 * n; ++k) dr[k] = dr[k] + (ddt * z->v[k] + dt * dv[k]);
        z->dt[q] = z->dt[q] + ddt;
    }
    for (int k = 0; k < 3 * n; ++k) z->r[k] = z->r[k] + dt * z->v[k];
    z->t = z->t + dt;
}

/* Kick K(ds): dt = ds/(alpha U + gamma); v += dt a.  Tangent: d(dt) = -(dt/g) alpha dU. */
static int t_kick(tstate *z, tscratch *w, double ds) {
    const int n = z->n;
    double U;
    int rc = orc_force_tlm(n, z->m, z->r, z->G, z->nd, z->dr, w->a, &U, w->da, w->dU, z->nthreads);
    if (rc) return rc;
    double g = z->alpha * U + z->gamma;
    double dt = ds / g;
    for (int q = 0; q < z->nd; ++q) {
        double *dv = z->dv + (size_t)q * 3 * n, *da = w->da + (size_t)q * 3 * n;
        double ddt = -(dt / g) * (z->alpha * w->dU[q]);
        for (int k = 0; k < 3 * n; ++k) dv[k] = dv[k] + (ddt * w->a[k] + dt * da[k]);
    }
    for (int k = 0; k < 3 * n; ++k) z->v[k] = z->v[k] + dt * w->a[k];
    return ORC_OK;
}

/* Lagrange weights of the extrapolation to h = 0 in the variable h^2 with
 * nodes h_k = H/n_k, n_k = 2k (Sec. 2.3, 4.2): T_{k_fix,k_fix} = sum_k c_k T_{k,1},
 * c_k = prod_{j != k} n_k^2 / (n_k^2 - n_j^2). */
void orc_lagrange_weights(int kf, double *c) {
    for (int k = 0; k < kf; ++k) {
        double nk2 = (double)(2 * (k + 1)) * (double)(2 * (k + 1));
        double w = 1.0;
        for (int j = 0; j < kf; ++j) {
            if (j == k) continue;
            double nj2 = (double)(2 * (j + 1)) * (double)(2 * (j + 1));
            w = w * (nk2 / (nk2 - nj2));
        }
        c[k] = w;
    }
}

/* Tangent-linear model of the replay: from (x0, v0) at t0 and directions
 * (dx0, dv0) [nd][n][3], nsteps GBS steps of lengths H[k] (each: the k_fix
 * leapfrog divisions from the step's start state combined with the Lagrange
 * weights).  Returns the end state in x, v, *t_out and its tangents in
 * dx, dv [nd][n][3], dt [nd]. */
int orc_replay_tlm(int n, const double *m, double *x, double *v, double t0, int64_t nsteps, const double *H,
                   const orc_params *p, int nd, double *dx, double *dv, double *dt, double *t_out) {
    if (n < 2 || nd < 0 || nsteps < 0 || !H || p->beta != 0.0 || p->k_fix < 2 || p->k_fix > 32) return ORC_E_INVAL;
    const int kf = p->k_fix;
    const size_t S3 = 3 * (size_t)n, SD = (size_t)nd * S3;
    double c[32];
    orc_lagrange_weights(kf, c);
    /* start-of-step state (r0, v0, t) with tangents, one division's state,
     * and the weighted increments of the new state */
    double *r0 = (double *)calloc(S3, sizeof(double)), *v0 = (double *)calloc(S3, sizeof(double));
    double *r = (double *)calloc(S3, sizeof(double)), *vv = (double *)calloc(S3, sizeof(double));
    double *ar = (double *)calloc(S3, sizeof(double)), *av = (double *)calloc(S3, sizeof(double));
    double *vc = (double *)calloc(S3, sizeof(double)), *acc = (double *)calloc(S3, sizeof(double));
    double *dr0 = (double *)calloc(SD + 1, sizeof(double)), *dv0 = (double *)calloc(SD + 1, sizeof(double));
    double *drr = (double *)calloc(SD + 1, sizeof(double)), *dvv = (double *)calloc(SD + 1, sizeof(double));
    double *adr = (double *)calloc(SD + 1, sizeof(double)), *adv = (double *)calloc(SD + 1, sizeof(double));
    double *da = (double *)calloc(SD + 1, sizeof(double));
    double *dt0 = (double *)calloc((size_t)nd + 1, sizeof(double)), *dtt = (double *)calloc((size_t)nd + 1, sizeof(double));
    double *adt = (double *)calloc((size_t)nd + 1, sizeof(double)), *dU = (double *)calloc((size_t)nd + 1, sizeof(double));
    double *dBv = (double *)calloc((size_t)nd + 1, sizeof(double));
    int rc = ORC_OK;
    if (!r0 || !v0 || !r || !vv || !ar || !av || !vc || !acc || !dr0 || !dv0 || !drr || !dvv || !adr || !adv ||
        !da || !dt0 || !dtt || !adt || !dU || !dBv) {
        rc = ORC_E_NOMEM;
        goto out;
    }
    tscratch w = {vc, acc, da, dU};
    memcpy(r0, x, sizeof(double) * S3);
    memcpy(v0, v, sizeof(double) * S3);
    memcpy(dr0, dx, sizeof(double) * SD);
    memcpy(dv0, dv, sizeof(double) * SD);
    double tt0 = t0, B;
    {   /* B = U(r0) - T(v0) and its tangent */
        tstate z = {n, nd, p->nthreads, m, p->G, p->alpha, p->gamma, 0.0, t0, r0, v0, dr0, dv0, dt0, dBv};
        double U;
        rc = orc_force_tlm(n, m, r0, p->G, nd, dr0, acc, &U, NULL, NULL, p->nthreads);
        if (rc) goto out;
        double T = t_kinetic(&z, vc);
        B = U - T;
        for (int q = 0; q < nd; ++q) {
            nsum s;
            ns_init(&s);
            const double *e = dr0 + (size_t)q * S3, *f = dv0 + (size_t)q * S3;
            for (int i = 0; i < n; ++i)
                for (int cc = 0; cc < 3; ++cc) {
                    ns_add(&s, m[i] * (acc[3 * i + cc] * e[3 * i + cc]));
                    ns_add(&s, -(m[i] * (vc[3 * i + cc] * f[3 * i + cc])));
                }
            dBv[q] = ns_get(&s);
        }
    }
    for (int64_t st = 0; st < nsteps; ++st) {
        /* accumulated increments of the new state */
        memset(ar, 0, sizeof(double) * S3); memset(av, 0, sizeof(double) * S3);
        memset(adr, 0, sizeof(double) * SD); memset(adv, 0, sizeof(double) * SD);
        double at = 0.0;
        for (int q = 0; q < nd; ++q) adt[q] = 0.0;
        for (int k = 0; k < kf; ++k) {
            memcpy(r, r0, sizeof(double) * S3); memcpy(vv, v0, sizeof(double) * S3);
            memcpy(drr, dr0, sizeof(double) * SD); memcpy(dvv, dv0, sizeof(double) * SD);
            memcpy(dtt, dt0, sizeof(double) * (size_t)nd);
            tstate z = {n, nd, p->nthreads, m, p->G, p->alpha, p->gamma, B, tt0, r, vv, drr, dvv, dtt, dBv};
            const int ns = 2 * (k + 1);
            const double h = H[st] / (double)ns;
            t_drift(&z, &w, 0.5 * h);
            for (int j = 0; j < ns - 1; ++j) {
                if ((rc = t_kick(&z, &w, h))) goto out;
                t_drift(&z, &w, h);
            }
            if ((rc = t_kick(&z, &w, h))) goto out;
            t_drift(&z, &w, 0.5 * h);
            /* increments from the start state, weighted */
            for (size_t i = 0; i < S3; ++i) { ar[i] += c[k] * (r[i] - r0[i]); av[i] += c[k] * (vv[i] - v0[i]); }
            for (size_t i = 0; i < SD; ++i) { adr[i] += c[k] * (drr[i] - dr0[i]); adv[i] += c[k] * (dvv[i] - dv0[i]); }
            at += c[k] * (z.t - tt0);
            for (int q = 0; q < nd; ++q) adt[q] += c[k] * (dtt[q] - dt0[q]);
        }
        for (size_t i = 0; i < S3; ++i) { r0[i] += ar[i]; v0[i] += av[i]; }
        for (size_t i = 0; i < SD; ++i) { dr0[i] += adr[i]; dv0[i] += adv[i]; }
        tt0 += at;
        for (int q = 0; q < nd; ++q) dt0[q] += adt[q];
    }
    memcpy(x, r0, sizeof(double) * S3);
    memcpy(v, v0, sizeof(double) * S3);
    memcpy(dx, dr0, sizeof(double) * SD);
    memcpy(dv, dv0, sizeof(double) * SD);
    for (int q = 0; q < nd; ++q) dt[q] = dt0[q];
    if (t_out) *t_out = tt0;
    rc = ORC_OK;
out:
    free(r0); free(v0); free(r); free(vv); free(ar); free(av); free(vc); free(acc);
    free(dr0); free(dv0); free(drr); free(dvv); free(adr); free(adv); free(da);
    free(dt0); free(dtt); free(adt); free(dU); free(dBv);
    return rc;
}

/* ------------------------------------------------------------------ */
/* Coordinate round trips (Sec. 3.5): the chained coordinates of Sec. 2.2 and
 * the repeated build / deconstruct cycle that compares them with the MST. */

/* Greedy chain (Sec. 2.2): the two ends of the shortest edge start the chain;
 * then the body outside the chain nearest to either end joins at that end,
 * until every body is in.  READINGS: edges and candidates are compared under
 * the strict order (w, min index, max index) of the MST; the lower-indexed end
 * of the first edge starts as the tail.  The chain is returned as a tree rooted
 * at its final tail: parent[] points one step towards the tail, level[] is the
 * distance from it, order[] lists the chain from tail to head. */
int orc_chain_build(int n, const double *x, int *parent, int *level, int *order) {
    if (n < 2) return ORC_E_INVAL;
    int a = 0, b = 1;
    double bw = edge_w(x, x + 3);
    for (int i = 0; i < n; ++i)
        for (int j = i + 1; j < n; ++j) {
            double w = edge_w(x + 3 * i, x + 3 * j);
            if (key_less(w, i, j, bw, a, b)) { bw = w; a = i; b = j; }
        }
    /* the chain as a deque in a buffer of 2n slots, tail at lo, head at hi - 1 */
    int *dq = (int *)malloc(sizeof(int) * 2 * (size_t)n);
    char *in = (char *)calloc((size_t)n, 1);
    if (!dq || !in) { free(dq); free(in); return ORC_E_NOMEM; }
    int lo = n, hi = n;
    dq[hi++] = a;
    dq[hi++] = b;
    in[a] = in[b] = 1;
    for (int added = 2; added < n; ++added) {
        const int tail = dq[lo], head = dq[hi - 1];
        int pick = -1, at_tail = 0;
        double pw = 0.0;
        int pend = -1;
        for (int u = 0; u < n; ++u) {
            if (in[u]) continue;
            const double wt = edge_w(x + 3 * tail, x + 3 * u), wh = edge_w(x + 3 * head, x + 3 * u);
            /* this body's nearer end, then the best body over all */
            int e = tail;
            double w = wt;
            if (key_less(wh, head, u, wt, tail, u)) { e = head; w = wh; }
            if (pick < 0 || key_less(w, e, u, pw, pend, pick)) { pick = u; pw = w; pend = e; at_tail = (e == tail); }
        }
        in[pick] = 1;
        if (at_tail) dq[--lo] = pick;
        else dq[hi++] = pick;
    }
    for (int k = 0; k < n; ++k) {
        const int v = dq[lo + k];
        order[k] = v;
        level[v] = k;
        parent[v] = k == 0 ? -1 : dq[lo + k - 1];
    }
    free(dq);
    free(in);
    return ORC_OK;
}

/* The rebuild test of Sec. 3.5: n_cycles times build the coordinate structure
 * from the Cartesian state (kind 0: MST rooted at the body nearest the centre of
 * mass, Sec. 3.2; kind 1: the chain above), form the edge vectors
 * X_v = x_v - x_parent(v), V_v likewise and the centre of mass, and deconstruct
 * back to Cartesian coordinates, x = r_cm + (rho - rho_bar).  Centre-of-mass
 * sums are compensated (Neumaier) unless kind has bit 2 set (kinds 2, 3):
 * then they are plain sums in index order, as the paper's test has them (Sec.
 * 3.5 leaves compensated summation for future work).  The physical state
 * does not change; only rounding accumulates.  x, v are updated in place; after
 * cycle (k+1) n_cycles / n_out (k < n_out) the state is copied to
 * xs[k], vs[k] ([n_out][n][3]).  levels_sum (nullable) receives the sum over
 * cycles of the mean level of the structure. */
int orc_rebuild_cycles(int n, const double *m, double *x, double *v, int kind, int64_t n_cycles, int n_out,
                       double *xs, double *vs, double *levels_sum) {
    if (n < 2 || kind < 0 || kind > 3 || n_cycles < 0 || n_out < 0 || (n_out > 0 && (!xs || !vs)))
        return ORC_E_INVAL;
    const int chain = kind & 1, plain = (kind & 2) != 0;
    void (*com)(int, const double *, const double *, double *) = plain ? com3_plain : com3;
    double *rho = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    if (!rho) return ORC_E_NOMEM;
    int *parent = (int *)malloc(sizeof(int) * (size_t)n), *level = (int *)malloc(sizeof(int) * (size_t)n);
    int *order = (int *)malloc(sizeof(int) * (size_t)n);
    double *X = (double *)malloc(sizeof(double) * 3 * (size_t)n), *V = (double *)malloc(sizeof(double) * 3 * (size_t)n);
    if (!parent || !level || !order || !X || !V) {
        free(parent); free(level); free(order); free(X); free(V); free(rho);
        return ORC_E_NOMEM;
    }
    int rc = ORC_OK, k = 0;
    double lsum = 0.0;
    for (int64_t cyc = 1; cyc <= n_cycles && !rc; ++cyc) {
        if (!chain) rc = orc_mst_prim(n, x, orc_root_nearest_com(n, m, x), parent, level, order);
        else rc = orc_chain_build(n, x, parent, level, order);
        if (rc) break;
        double ls = 0.0;
        for (int u = 0; u < n; ++u) ls += level[u];
        lsum += ls / n;
        double scal[9];
        for (int u = 0; u < n; ++u) {
            const int q = parent[u];
            for (int c = 0; c < 3; ++c) {
                X[3 * u + c] = q < 0 ? 0.0 : x[3 * u + c] - x[3 * q + c];
                V[3 * u + c] = q < 0 ? 0.0 : v[3 * u + c] - v[3 * q + c];
            }
        }
        com(n, m, x, scal + 3);
        com(n, m, v, scal + 6);
        /* x = r_cm + (rho - rho_bar), v alike (rho: top-down path sums) */
        for (int pass = 0; pass < 2; ++pass) {
            double c[3];
            orc_deconstruct(n, parent, order, pass ? V : X, rho);
            com(n, m, rho, c);
            double *out = pass ? v : x;
            for (int i = 0; i < n; ++i)
                for (int k = 0; k < 3; ++k) out[3 * i + k] = scal[(pass ? 6 : 3) + k] + (rho[3 * i + k] - c[k]);
        }
        while (!rc && k < n_out && cyc == ((int64_t)(k + 1) * n_cycles) / n_out) {
            memcpy(xs + (size_t)k * 3 * n, x, sizeof(double) * 3 * (size_t)n);
            memcpy(vs + (size_t)k * 3 * n, v, sizeof(double) * 3 * (size_t)n);
            ++k;
        }
    }
    if (levels_sum) *levels_sum = lsum;
    free(parent); free(level); free(order); free(X); free(V); free(rho);
    return rc;
}
