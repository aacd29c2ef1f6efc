// Minimum spanning tree and tree transforms on the GPU (paper Sec. 3.1-3.5).
//
//  * Tree sums (deconstruction, Sec. 2.2/3.4): root-relative positions
//    rho_v = sum of the edge vectors on the root -> v path, by pointer jumping
//    (ceil(log2 depth) rounds) in one workgroup.
//  * MST: Boruvka rounds on the complete graph under the strict edge order
//    (w = (dx*dx + dy*dy) + dz*dz without FMA, min index, max index), which
//    yields the unique MST of Sec. 3.1 -- the same tree Prim's algorithm of
//    Sec. 3.2 finds.  The O(N^2) scan of each round runs on the whole chip
//    (scalar-loaded j-bodies, one i per lane); the per-component minimum,
//    hooking and pointer-jumping contraction run in one workgroup.
//  * Rooting at the body nearest the centre of mass (Sec. 3.2) with an Euler
//    tour and list ranking (O(log N) rounds), giving parent and level
//    (Sec. 3.4) and children lists for the close-pair rule.
//  * Rebuild (Sec. 3.5): each new edge vector is the separation the previous
//    tree gives for that pair under the close-pair rule (an edge that
//    persists keeps its bits; a reversed edge is negated exactly).
#include "common.h"

namespace mstar {

// ------------------------------------------------------------ tree sums
__global__ __launch_bounds__(kTreeWG) void k_tree_sums(Dev d, const d4 *X, const d4 *V, d4 *rho, d4 *ups) {
    __shared__ int any;
    const int n = d.n;
    d4 *SX[2] = {d.tsC, d.tsD};
    d4 *SV[2] = {d.tsE, d.tsF};
    int32_t *anc[2] = {d.ancA, d.ancB};
    for (int v = threadIdx.x; v < n; v += kTreeWG) {
        const int a = d.parent[v];
        SX[0][v] = a < 0 ? d4{0.0, 0.0, 0.0, 0.0} : X[v];
        SV[0][v] = a < 0 ? d4{0.0, 0.0, 0.0, 0.0} : V[v];
        anc[0][v] = a;
    }
    int cur = 0;
    for (int it = 0; it < 64; ++it) {   // 2^64 exceeds any list: bounded
        if (threadIdx.x == 0) any = 0;
        __threadfence_block();
        __syncthreads();
        const int nx = cur ^ 1;
        for (int v = threadIdx.x; v < n; v += kTreeWG) {
            const int a = anc[cur][v];
            if (a >= 0) {
                const d4 x = SX[cur][v], xa = SX[cur][a], w = SV[cur][v], wa = SV[cur][a];
                SX[nx][v] = d4{x.x + xa.x, x.y + xa.y, x.z + xa.z, 0.0};
                SV[nx][v] = d4{w.x + wa.x, w.y + wa.y, w.z + wa.z, 0.0};
                const int aa = anc[cur][a];
                anc[nx][v] = aa;
                if (aa >= 0) any = 1;
            } else {
                SX[nx][v] = SX[cur][v];
                SV[nx][v] = SV[cur][v];
                anc[nx][v] = -1;
            }
        }
        __threadfence_block();
        __syncthreads();
        cur = nx;
        const int a2 = any;
        __syncthreads();
        if (!a2) break;
    }
    for (int v = threadIdx.x; v < n; v += kTreeWG) {
        rho[v] = SX[cur][v];
        ups[v] = SV[cur][v];
    }
}

void launch_tree_sums(const Dev &d, hipStream_t s, const d4 *X, const d4 *V, d4 *rho, d4 *ups) {
    k_tree_sums<<<1, kTreeWG, 0, s>>>(d, X, V, rho, ups);
}

// ------------------------------------------------------------ MST
__device__ __forceinline__ double mst_w(const d4 &a, const d4 &b) {
    const double dx = b.x - a.x, dy = b.y - a.y, dz = b.z - a.z;
    return (dx * dx + dy * dy) + dz * dz;   // no contraction (-ffp-contract=off)
}

// Root choice (Sec. 3.2): nearest to the centre of mass, ties to the lowest
// index; resets the Boruvka components.
__global__ __launch_bounds__(kTreeWG) void k_mst_init(Dev d, const d4 *pos, int root_in) {
    __shared__ double sh[kTreeWG];
    __shared__ double sw[kTreeWG];
    __shared__ int si[kTreeWG];
    const int n = d.n;
    for (int v = threadIdx.x; v < n; v += kTreeWG) {
        d.comp[v] = v;
        d.hooked[v] = 0;
    }
    if (threadIdx.x == 0) {
        *d.done = 0;
        *d.ncomp = n;
    }
    if (root_in >= 0 && root_in < n) {
        if (threadIdx.x == 0) *d.root = root_in;
        return;
    }
    double sm = 0.0, s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int v = threadIdx.x; v < n; v += kTreeWG) {
        const double mu = d.m[v];
        const d4 p = pos[v];
        sm = sm + mu;
        s0 = s0 + mu * p.x; s1 = s1 + mu * p.y; s2 = s2 + mu * p.z;
    }
    const double M = block_sum<kTreeWG>(sm, sh);
    const d4 c{block_sum<kTreeWG>(s0, sh) / M, block_sum<kTreeWG>(s1, sh) / M, block_sum<kTreeWG>(s2, sh) / M, 0.0};
    double bw = INFINITY;
    int bi = 0x7fffffff;
    for (int v = threadIdx.x; v < n; v += kTreeWG) {
        const double w = mst_w(c, pos[v]);
        if (w < bw) { bw = w; bi = v; }
    }
    sw[threadIdx.x] = bw;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int s = kTreeWG / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const double w2 = sw[threadIdx.x + s];
            const int i2 = si[threadIdx.x + s];
            if (w2 < sw[threadIdx.x] || (w2 == sw[threadIdx.x] && i2 < si[threadIdx.x])) {
                sw[threadIdx.x] = w2;
                si[threadIdx.x] = i2;
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) *d.root = si[0];
}

// One Boruvka scan: for every body i the lightest edge (w, j) to a body of
// another component, over the workgroup's j-range (j ascending per lane, so
// equal weights keep the smaller j, i.e. the strict order for fixed i).
__global__ __launch_bounds__(256) void k_bor_scan(Dev d, const d4 *__restrict__ pos, int nsplit, int jchunk) {
    if (*d.done) return;
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int n = d.n;
    const int i = blockIdx.x * 64 + lane;
    const int ii = i < n ? i : n - 1;
    const d4 pi = pos[ii];
    const int32_t *__restrict__ comp = d.comp;
    const int ci = comp[ii];
    const int j0 = blockIdx.y * jchunk;
    const int j1 = min(n, j0 + jchunk);
    const int q = (max(j1 - j0, 0) + 3) >> 2;
    int jb = min(j1, j0 + wv * q);
    int je = min(j1, jb + q);
    jb = __builtin_amdgcn_readfirstlane(jb);
    je = __builtin_amdgcn_readfirstlane(je);
    double bw = INFINITY;
    int bj = -1;
#pragma unroll 4
    for (int j = jb; j < je; ++j) {
        const d4 pj = pos[j];
        const int cj = comp[j];
        const double w = mst_w(pi, pj);
        const bool take = (cj != ci) && (w < bw);
        bw = take ? w : bw;
        bj = take ? j : bj;
    }
    __shared__ double rw[4][64];
    __shared__ int rj[4][64];
    rw[wv][lane] = bw;
    rj[wv][lane] = bj;
    __syncthreads();
    if (wv != 0 || i >= n) return;
    for (int w = 1; w < 4; ++w) {
        const double w2 = rw[w][lane];
        const int j2 = rj[w][lane];
        if (j2 >= 0 && (bj < 0 || w2 < bw || (w2 == bw && j2 < bj))) { bw = w2; bj = j2; }
    }
    d.bor_w[(size_t)blockIdx.y * n + i] = bw;
    d.bor_j[(size_t)blockIdx.y * n + i] = bj;
}

// Component minimum, hooking and contraction (one workgroup).
__global__ __launch_bounds__(kTreeWG) void k_bor_merge(Dev d, int nsplit) {
    __shared__ int changed;
    __shared__ int cnt;
    if (*d.done) return;
    const int n = d.n;
    double *mw = d.scr;                 // [n]
    int32_t *mj = d.ecomp_tmp;          // [n]
    for (int i = threadIdx.x; i < n; i += kTreeWG) {
        double bw = INFINITY;
        int bj = -1;
        for (int s = 0; s < nsplit; ++s) {
            const double w2 = d.bor_w[(size_t)s * n + i];
            const int j2 = d.bor_j[(size_t)s * n + i];
            if (j2 >= 0 && (bj < 0 || w2 < bw || (w2 == bw && j2 < bj))) { bw = w2; bj = j2; }
        }
        mw[i] = bw;
        mj[i] = bj;
        if (d.comp[i] == i) {
            d.cw[i] = ~0ull;
            d.cidx[i] = ~0ull;
        }
    }
    __threadfence_block();
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += kTreeWG)
        if (mj[i] >= 0) atomicMin(&d.cw[d.comp[i]], (unsigned long long)__double_as_longlong(mw[i]));
    __threadfence_block();
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += kTreeWG) {
        const int j = mj[i];
        if (j >= 0 && (unsigned long long)__double_as_longlong(mw[i]) == d.cw[d.comp[i]]) {
            const unsigned long long lo = (unsigned)min(i, j), hi = (unsigned)max(i, j);
            atomicMin(&d.cidx[d.comp[i]], (lo << 32) | hi);
        }
    }
    __threadfence_block();
    __syncthreads();
    for (int c = threadIdx.x; c < n; c += kTreeWG) {
        if (d.comp[c] != c) continue;
        const unsigned long long k = d.cidx[c];
        if (k == ~0ull) { d.tgt[c] = c; continue; }
        const int lo = (int)(k >> 32), hi = (int)(k & 0xffffffffull);
        const int other = (d.comp[lo] == c) ? hi : lo;
        d.tgt[c] = d.comp[other];
        d.elo[c] = lo;
        d.ehi[c] = hi;
    }
    __threadfence_block();
    __syncthreads();
    // hook: a mutual pair keeps the smaller id as representative; every hook
    // records its edge at the index of the hooking representative
    for (int c = threadIdx.x; c < n; c += kTreeWG) {
        if (d.comp[c] != c) continue;
        const int t = d.tgt[c];
        if (t == c) continue;
        if (d.tgt[t] == c && c < t) continue;
        d.hooked[c] = 1;
        d.ecomp_tmp[c] = t;   // new representative (mj no longer needed for roots)
    }
    __threadfence_block();
    __syncthreads();
    for (int c = threadIdx.x; c < n; c += kTreeWG)
        if (d.comp[c] == c && d.hooked[c] && d.tgt[c] != c && !(d.tgt[d.tgt[c]] == c && c < d.tgt[c]))
            d.comp[c] = d.ecomp_tmp[c];
    __threadfence_block();
    __syncthreads();
    for (int it = 0; it < 64; ++it) {   // 2^64 exceeds any list: bounded
        if (threadIdx.x == 0) changed = 0;
        __syncthreads();
        for (int v = threadIdx.x; v < n; v += kTreeWG) {
            const int c = d.comp[v];
            const int cc = d.comp[c];
            if (cc != c) { d.comp[v] = cc; changed = 1; }
        }
        __threadfence_block();
        __syncthreads();
        const int ch = changed;
        __syncthreads();
        if (!ch) break;
    }
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    int local = 0;
    for (int v = threadIdx.x; v < n; v += kTreeWG) local += (d.comp[v] == v);
    atomicAdd(&cnt, local);
    __syncthreads();
    if (threadIdx.x == 0) {
        *d.ncomp = cnt;
        if (cnt <= 1) *d.done = 1;
    }
}

// Exclusive prefix sum of in[0..n) into out[0..n], one workgroup.
__device__ void block_scan_excl(const int32_t *in, int32_t *out, int n, int *sh) {
    const int t = threadIdx.x;
    const int chunk = (n + kTreeWG - 1) / kTreeWG;
    const int b = min(n, t * chunk), e = min(n, b + chunk);
    int loc = 0;
    for (int k = b; k < e; ++k) loc += in[k];
    sh[t] = loc;
    __syncthreads();
    for (int off = 1; off < kTreeWG; off <<= 1) {
        const int add = (t >= off) ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += add;
        __syncthreads();
    }
    int run = sh[t] - loc;
    for (int k = b; k < e; ++k) {
        const int x = in[k];
        out[k] = run;
        run += x;
    }
    if (t == kTreeWG - 1) out[n] = sh[t];
    __threadfence_block();
    __syncthreads();
}

// Levels by pointer jumping over parents, children lists sorted by index.
__device__ void levels_and_children(Dev &d, const int32_t *par, int32_t *lev, int *sh) {
    __shared__ int any;
    const int n = d.n;
    int32_t *L[2] = {d.rkA, d.rkB};
    int32_t *A[2] = {d.nxtA, d.nxtB};
    for (int v = threadIdx.x; v < n; v += kTreeWG) {
        L[0][v] = par[v] < 0 ? 0 : 1;
        A[0][v] = par[v];
        d.cnt[v] = 0;
    }
    __threadfence_block();
    __syncthreads();
    int cur = 0;
    for (int it = 0; it < 64; ++it) {   // 2^64 exceeds any list: bounded
        if (threadIdx.x == 0) any = 0;
        __syncthreads();
        const int nx = cur ^ 1;
        for (int v = threadIdx.x; v < n; v += kTreeWG) {
            const int a = A[cur][v];
            if (a >= 0) {
                L[nx][v] = L[cur][v] + L[cur][a];
                const int aa = A[cur][a];
                A[nx][v] = aa;
                if (aa >= 0) any = 1;
            } else {
                L[nx][v] = L[cur][v];
                A[nx][v] = -1;
            }
        }
        __threadfence_block();
        __syncthreads();
        cur = nx;
        const int a2 = any;
        __syncthreads();
        if (!a2) break;
    }
    for (int v = threadIdx.x; v < n; v += kTreeWG) {
        lev[v] = L[cur][v];
        if (par[v] >= 0) atomicAdd(&d.cnt[par[v]], 1);
    }
    __threadfence_block();
    __syncthreads();
    block_scan_excl(d.cnt, d.child_off, n, sh);
    for (int v = threadIdx.x; v < n; v += kTreeWG) d.fill[v] = 0;
    __threadfence_block();
    __syncthreads();
    for (int v = threadIdx.x; v < n; v += kTreeWG) {
        const int p = par[v];
        if (p >= 0) d.child_idx[d.child_off[p] + atomicAdd(&d.fill[p], 1)] = v;
    }
    __threadfence_block();
    __syncthreads();
    for (int v = threadIdx.x; v < n; v += kTreeWG) {   // insertion sort of each (short) list
        const int b = d.child_off[v], e = d.child_off[v + 1];
        for (int k = b + 1; k < e; ++k) {
            const int x = d.child_idx[k];
            int q = k - 1;
            while (q >= b && d.child_idx[q] > x) { d.child_idx[q + 1] = d.child_idx[q]; --q; }
            d.child_idx[q + 1] = x;
        }
    }
    __threadfence_block();
    __syncthreads();
}

// Root the MST at *d.root with an Euler tour: arc 2c = lo->hi, 2c+1 = hi->lo
// for every hooked c; the successor of arc u->v is the arc after v->u in v's
// cyclic adjacency list; ranks by pointer jumping; an edge's first-traversed
// arc points from the parent to the child.  Writes parent_new, level_new and
// the children lists.
__global__ __launch_bounds__(kTreeWG) void k_root_tree(Dev d) {
    __shared__ int sh[kTreeWG];
    __shared__ int any;
    __shared__ int last;
    const int n = d.n;
    const int root = *d.root;
    for (int v = threadIdx.x; v < n; v += kTreeWG) {
        d.deg[v] = 0;
        d.fill[v] = 0;
    }
    __threadfence_block();
    __syncthreads();
    for (int c = threadIdx.x; c < n; c += kTreeWG)
        if (d.hooked[c]) {
            atomicAdd(&d.deg[d.elo[c]], 1);
            atomicAdd(&d.deg[d.ehi[c]], 1);
        }
    __threadfence_block();
    __syncthreads();
    block_scan_excl(d.deg, d.off, n, sh);
    for (int c = threadIdx.x; c < n; c += kTreeWG)
        if (d.hooked[c]) {
            const int lo = d.elo[c], hi = d.ehi[c];
            const int s0 = d.off[lo] + atomicAdd(&d.fill[lo], 1);
            d.adj[s0] = 2 * c;
            d.arcpos[2 * c] = s0;
            const int s1 = d.off[hi] + atomicAdd(&d.fill[hi], 1);
            d.adj[s1] = 2 * c + 1;
            d.arcpos[2 * c + 1] = s1;
        }
    __threadfence_block();
    __syncthreads();
    const int first = d.adj[d.off[root]];
    if (threadIdx.x == 0) last = -1;
    for (int a = threadIdx.x; a < 2 * n; a += kTreeWG) {
        const int c = a >> 1;
        if (!d.hooked[c]) { d.nxtA[a] = -2; continue; }
        const int v = (a & 1) ? d.elo[c] : d.ehi[c];     // destination of arc a
        const int p = d.arcpos[a ^ 1];
        int q = p + 1;
        if (q == d.off[v + 1]) q = d.off[v];
        d.nxtA[a] = d.adj[q];
    }
    __threadfence_block();
    __syncthreads();
    for (int a = threadIdx.x; a < 2 * n; a += kTreeWG)
        if (d.nxtA[a] == first) last = a;
    __syncthreads();
    if (threadIdx.x == 0 && last >= 0) d.nxtA[last] = -1;
    __threadfence_block();
    __syncthreads();
    int32_t *R[2] = {d.rkA, d.rkB};
    int32_t *N[2] = {d.nxtA, d.nxtB};
    for (int a = threadIdx.x; a < 2 * n; a += kTreeWG) R[0][a] = (N[0][a] >= 0) ? 1 : 0;
    __threadfence_block();
    __syncthreads();
    int cur = 0;
    for (int it = 0; it < 64; ++it) {   // 2^64 exceeds any list: bounded
        if (threadIdx.x == 0) any = 0;
        __syncthreads();
        const int nx = cur ^ 1;
        for (int a = threadIdx.x; a < 2 * n; a += kTreeWG) {
            const int b = N[cur][a];
            if (b >= 0) {
                R[nx][a] = R[cur][a] + R[cur][b];
                const int bb = N[cur][b];
                N[nx][a] = bb;
                if (bb >= 0) any = 1;
            } else {
                R[nx][a] = R[cur][a];
                N[nx][a] = b;
            }
        }
        __threadfence_block();
        __syncthreads();
        cur = nx;
        const int a2 = any;
        __syncthreads();
        if (!a2) break;
    }
    int32_t *rank = R[cur];
    for (int c = threadIdx.x; c < n; c += kTreeWG) {
        if (!d.hooked[c]) continue;
        const int lo = d.elo[c], hi = d.ehi[c];
        if (rank[2 * c] > rank[2 * c + 1]) d.parent_new[hi] = lo;
        else d.parent_new[lo] = hi;
    }
    if (threadIdx.x == 0) d.parent_new[root] = -1;
    __threadfence_block();
    __syncthreads();
    levels_and_children(d, d.parent_new, d.level_new, sh);
}

int launch_mst(const Dev &d, hipStream_t s, const d4 *pos, int root_in, int nsplit) {
    k_mst_init<<<1, kTreeWG, 0, s>>>(d, pos, root_in);
    const int jchunk = (d.n + nsplit - 1) / nsplit;
    int rounds = 0;
    for (int m = 1; m < d.n; m <<= 1) ++rounds;   // components at least halve per round
    for (int r = 0; r < rounds; ++r) {
        k_bor_scan<<<dim3(d.nib, nsplit), 256, 0, s>>>(d, pos, nsplit, jchunk);
        k_bor_merge<<<1, kTreeWG, 0, s>>>(d, nsplit);
    }
    k_root_tree<<<1, kTreeWG, 0, s>>>(d);
    return rounds;
}

// Levels and children of the current tree (parent[]), for stage calls that
// receive a tree from the caller.
__global__ __launch_bounds__(kTreeWG) void k_levels_children(Dev d) {
    __shared__ int sh[kTreeWG];
    levels_and_children(d, d.parent, d.level, sh);
}

void launch_levels_children(const Dev &d, hipStream_t s) { k_levels_children<<<1, kTreeWG, 0, s>>>(d); }

// ------------------------------------------------------------ rebuild
// Separation d_ij under the close-pair rule of the (old) tree: the path sum
// S_j - S_i through the lowest common ancestor when the tree distance is at
// most nd (eq. LCA), else rho_j - rho_i.
__device__ d4 sep_rule(int i, int j, const int32_t *par, const int32_t *lev, const d4 *X, const d4 *rho, int nd) {
    if (i != j && nd > 0 && abs(lev[i] - lev[j]) <= nd) {
        int anc[8];
        int na = 0, u = i;
        for (int a = 0; a <= nd; ++a) {
            anc[na++] = u;
            if (par[u] < 0) break;
            u = par[u];
        }
        int w = j, fa = -1, fb = -1;
        for (int b = 0; b <= nd && fa < 0; ++b) {
            for (int a = 0; a < na && a + b <= nd; ++a)
                if (anc[a] == w) { fa = a; fb = b; break; }
            if (fa >= 0 || par[w] < 0) break;
            w = par[w];
        }
        if (fa >= 0) {
            d4 si{0.0, 0.0, 0.0, 0.0}, sj{0.0, 0.0, 0.0, 0.0};
            int pth[8];
            u = i;
            for (int s = 0; s < fa; ++s) { pth[s] = u; u = par[u]; }
            for (int s = fa - 1; s >= 0; --s) { const d4 x = X[pth[s]]; si.x = si.x + x.x; si.y = si.y + x.y; si.z = si.z + x.z; }
            u = j;
            for (int s = 0; s < fb; ++s) { pth[s] = u; u = par[u]; }
            for (int s = fb - 1; s >= 0; --s) { const d4 x = X[pth[s]]; sj.x = sj.x + x.x; sj.y = sj.y + x.y; sj.z = sj.z + x.z; }
            return d4{sj.x - si.x, sj.y - si.y, sj.z - si.z, 0.0};
        }
    }
    const d4 a = rho[i], b = rho[j];
    return d4{b.x - a.x, b.y - a.y, b.z - a.z, 0.0};
}

__global__ __launch_bounds__(kWG) void k_rebuild_edges(Dev d, const d4 *rho, const d4 *ups, int nd) {
    const int n = d.n;
    const int u = blockIdx.x * kWG + threadIdx.x;
    if (u >= n) return;
    const int q = d.parent_new[u];
    d4 X{0.0, 0.0, 0.0, 0.0}, V{0.0, 0.0, 0.0, 0.0};
    if (q >= 0) {
        X = sep_rule(q, u, d.parent, d.level, d.X0, rho, nd);
        V = sep_rule(q, u, d.parent, d.level, d.V0, ups, nd);
    }
    d.tsC[u] = X;
    d.tsD[u] = V;
    if (q != d.parent[u]) d.ctl->topo = 1;
}

__global__ __launch_bounds__(kWG) void k_swap_tree(Dev d) {
    const int n = d.n;
    const int u = blockIdx.x * kWG + threadIdx.x;
    if (u >= n) return;
    d.X0[u] = d.tsC[u];
    d.V0[u] = d.tsD[u];
    d.parent[u] = d.parent_new[u];
    d.level[u] = d.level_new[u];
}

__global__ void k_zero_counter(Dev d) { d.ctl->topo = 0; }

void launch_rebuild_edges(const Dev &d, hipStream_t s, const d4 *rho, const d4 *ups, int nd) {
    const int nb = (d.n + kWG - 1) / kWG;
    k_zero_counter<<<1, 1, 0, s>>>(d);
    k_rebuild_edges<<<nb, kWG, 0, s>>>(d, rho, ups, nd);
    k_swap_tree<<<nb, kWG, 0, s>>>(d);
}

__global__ __launch_bounds__(kWG) void k_adopt_tree(Dev d) {
    const int u = blockIdx.x * kWG + threadIdx.x;
    if (u >= d.n) return;
    d.parent[u] = d.parent_new[u];
    d.level[u] = d.level_new[u];
}

void launch_tree_finish(const Dev &d, hipStream_t s) {
    k_adopt_tree<<<(d.n + kWG - 1) / kWG, kWG, 0, s>>>(d);
}

}  // namespace mstar
