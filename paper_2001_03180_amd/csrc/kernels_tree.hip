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
        d.cw[v] = ~0ull;
        d.cidx[v] = ~0ull;
        d.parent_new[v] = -1;
    }
    if (threadIdx.x == 0) {
        *d.done = 0;
        *d.ncomp = n;
        *d.rounds = 0;
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
    constexpr int W = kTreeWG / 64;
    const double M = block_sum1<kTreeWG>(sm, sh);
    const d4 c{block_sum1<kTreeWG>(s0, sh + W) / M, block_sum1<kTreeWG>(s1, sh + 2 * W) / M,
               block_sum1<kTreeWG>(s2, sh + 3 * W) / M, 0.0};
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
// another component over the workgroup's j-range (j ascending per lane, so
// equal weights keep the smaller j, i.e. the strict order for fixed i).
// Workgroup = 4 waves sharing 64 bodies, each a quarter of the j-range.
__global__ __launch_bounds__(256) void k_bor_scan(Dev d, const d4 *__restrict__ pos, int jchunk) {
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

// Per body: the best of the split results in (w, j) order (four threads per
// body, each a fixed quarter of the splits, combined in fixed order); the
// component's minimum weight is lowered with a 64-bit atomic on the weight bits.
__global__ __launch_bounds__(kWG) void k_bor_vreduce(Dev d, int nsplit) {
    if (*d.done) return;
    __shared__ double rw[kWG];
    __shared__ int rj[kWG];
    const int n = d.n;
    const int i = blockIdx.x * (kWG / 4) + (threadIdx.x >> 2);
    const int part = threadIdx.x & 3;
    double bw = INFINITY;
    int bj = -1;
    if (i < n) {
        for (int s = part; s < nsplit; s += 4) {
            const double w2 = d.bor_w[(size_t)s * n + i];
            const int j2 = d.bor_j[(size_t)s * n + i];
            if (j2 >= 0 && (bj < 0 || w2 < bw || (w2 == bw && j2 < bj))) { bw = w2; bj = j2; }
        }
    }
    rw[threadIdx.x] = bw;
    rj[threadIdx.x] = bj;
    __syncthreads();
    if (part != 0 || i >= n) return;
    for (int k = 1; k < 4; ++k) {
        const double w2 = rw[threadIdx.x + k];
        const int j2 = rj[threadIdx.x + k];
        if (j2 >= 0 && (bj < 0 || w2 < bw || (w2 == bw && j2 < bj))) { bw = w2; bj = j2; }
    }
    d.scr[i] = bw;
    d.ecomp_tmp[i] = bj;
    if (bj >= 0) {
        const unsigned long long key = (unsigned long long)__double_as_longlong(bw);
        unsigned long long *slot = &d.cw[d.comp[i]];
        if (key < __atomic_load_n(slot, __ATOMIC_RELAXED)) atomicMin(slot, key);   // skip hopeless atomics
    }
}

// Component minimum (tie-break on packed (min, max) indices), hooking with
// mutual pairs broken toward the smaller representative, contraction, and the
// count of components (one workgroup; component ids, hook pointers, the
// parent pointers and the per-component best edge in LDS when they fit).
//
// Parent pointers are maintained as the components grow: every component's
// edges point toward one of its bodies (its tree root).  When component c
// hooks onto another through the edge (a in c, b outside c), the parent
// pointers on the path from a to c's tree root are reversed and a points to
// b; the paths of different hooking components are disjoint, so all hooks of a
// round are applied in parallel.
template <bool LDS>
__global__ __launch_bounds__(kTreeWG) void k_bor_merge(Dev d) {
    extern __shared__ unsigned long long lds64[];
    __shared__ int cnt;
    if (*d.done) return;
    const int n = d.n;
    int *ib = reinterpret_cast<int *>(lds64 + n);   // LDS: n 64-bit keys, then 4n ints
    unsigned long long *cidx = LDS ? lds64 : d.cidx;
    int *comp = LDS ? ib : d.comp;
    int *hook = LDS ? ib + n : d.fill;
    int *tgt = LDS ? ib + 2 * n : d.tgt;
    int *par = LDS ? ib + 3 * n : d.parent_new;
    if (LDS) {
        for (int v = threadIdx.x; v < n; v += kTreeWG) {
            comp[v] = d.comp[v];
            par[v] = d.parent_new[v];
            cidx[v] = ~0ull;
        }
        __syncthreads();
    }
    const double *mw = d.scr;
    const int32_t *mj = d.ecomp_tmp;
    for (int i = threadIdx.x; i < n; i += kTreeWG) {
        const int j = mj[i];
        const int c = comp[i];
        if (j >= 0 && (unsigned long long)__double_as_longlong(mw[i]) == d.cw[c]) {
            const unsigned long long lo = (unsigned)min(i, j), hi = (unsigned)max(i, j);
            atomicMin(&cidx[c], (lo << 32) | hi);
        }
    }
    __threadfence_block();
    __syncthreads();
    for (int c = threadIdx.x; c < n; c += kTreeWG) {
        if (comp[c] != c) continue;
        const unsigned long long k = cidx[c];
        if (k == ~0ull) { tgt[c] = c; continue; }
        const int lo = (int)(k >> 32), hi = (int)(k & 0xffffffffull);
        const bool lo_in = (comp[lo] == c);
        tgt[c] = comp[lo_in ? hi : lo];
    }
    __threadfence_block();
    __syncthreads();
    // hook: every representative moves under its target except the smaller
    // member of a mutual pair; the hooking component re-roots at its end of
    // the edge and hangs from the other end
    for (int c = threadIdx.x; c < n; c += kTreeWG) {
        if (comp[c] != c) continue;
        const int t = tgt[c];
        if (t == c || (tgt[t] == c && c < t)) { hook[c] = c; continue; }
        hook[c] = t;
        // the edge's end inside c and the one outside it, again from the key
        const unsigned long long k = cidx[c];
        const int lo = (int)(k >> 32), hi = (int)(k & 0xffffffffull);
        const bool lo_in = (comp[lo] == c);
        int prev = lo_in ? hi : lo, x = lo_in ? lo : hi;
        for (int it = 0; it < n && x >= 0; ++it) {
            const int nx = par[x];
            par[x] = prev;
            prev = x;
            x = nx;
        }
    }
    __threadfence_block();
    __syncthreads();
    // contraction: follow the hook pointers of representatives to the root
    for (int v = threadIdx.x; v < n; v += kTreeWG) {
        int c = comp[v];
        for (int it = 0; it < n && hook[c] != c; ++it) c = hook[c];
        tgt[v] = c;   // tgt is free again
    }
    __threadfence_block();
    __syncthreads();
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    int local = 0;
    for (int v = threadIdx.x; v < n; v += kTreeWG) {
        const int c = tgt[v];
        d.comp[v] = c;
        if (LDS) d.parent_new[v] = par[v];
        if (c == v) {
            ++local;
            d.cw[v] = ~0ull;
            if (!LDS) d.cidx[v] = ~0ull;
        }
    }
    atomicAdd(&cnt, local);
    __syncthreads();
    if (threadIdx.x == 0) {
        *d.ncomp = cnt;
        *d.rounds += 1;
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

// Final rooting (Sec. 3.2: the body nearest the centre of mass): reverse the
// parent pointers on the path from the chosen root to the current tree root,
// then levels by pointer jumping (parent, grandparent, ...) and the children
// lists (ascending index) by counting, one workgroup with LDS when it fits.
constexpr int kFinWG = 1024;

template <bool LDS>
__global__ __launch_bounds__(kFinWG) void k_mst_finish(Dev d) {
    extern __shared__ int lds[];
    __shared__ int sh[kFinWG];
    __shared__ int any;
    // rounds launched without a host check may not have finished the tree:
    // then nothing is changed and the old tree stays (tree_bad)
    const int fin = *d.done;
    if (threadIdx.x == 0) {
        d.ctl->tree_bad = fin ? 0 : 1;
        if (fin) d.ctl->mst_rounds = *d.rounds;
    }
    if (!fin) return;
    const int n = d.n;
    const int root = *d.root;
    int *par = LDS ? lds : d.parent_new;          // n
    int *lev = LDS ? lds + n : d.level_new;       // n
    int *anc = LDS ? lds + 2 * n : d.deg;         // n
    int *cnt = LDS ? lds + 3 * n : d.off;         // n + 1
    if (LDS) {
        for (int v = threadIdx.x; v < n; v += kFinWG) par[v] = d.parent_new[v];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        int prev = -1, x = root;
        for (int it = 0; it < n && x >= 0; ++it) {
            const int nx = par[x];
            par[x] = prev;
            prev = x;
            x = nx;
        }
    }
    __threadfence_block();
    __syncthreads();
    for (int v = threadIdx.x; v < n; v += kFinWG) {
        lev[v] = par[v] < 0 ? 0 : 1;
        anc[v] = par[v];
        cnt[v] = 0;
    }
    if (threadIdx.x == 0) cnt[n] = 0;
    __threadfence_block();
    __syncthreads();
    // pointer jumping in place: read a thread's bodies into registers, barrier, write
    constexpr int kPer = 16;
    const bool fits = (n + kFinWG - 1) / kFinWG <= kPer;
    for (int it = 0; it < 64; ++it) {
        if (threadIdx.x == 0) any = 0;
        __syncthreads();
        if (fits) {
            int nl[kPer], na[kPer];
#pragma unroll
            for (int k = 0; k < kPer; ++k) {
                const int v = threadIdx.x + k * kFinWG;
                nl[k] = 0; na[k] = -1;
                if (v < n) {
                    const int a = anc[v];
                    nl[k] = lev[v];
                    if (a >= 0) {
                        nl[k] = lev[v] + lev[a];
                        na[k] = anc[a];
                        if (na[k] >= 0) any = 1;
                    }
                }
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < kPer; ++k) {
                const int v = threadIdx.x + k * kFinWG;
                if (v < n) { lev[v] = nl[k]; anc[v] = na[k]; }
            }
        } else {
            // large N: jump one body at a time through a private copy in global scratch
            for (int v = threadIdx.x; v < n; v += kFinWG) {
                const int a = anc[v];
                d.nxtA[v] = (a >= 0) ? lev[v] + lev[a] : lev[v];
                d.nxtB[v] = (a >= 0) ? anc[a] : -1;
                if (a >= 0 && anc[a] >= 0) any = 1;
            }
            __threadfence_block();
            __syncthreads();
            for (int v = threadIdx.x; v < n; v += kFinWG) { lev[v] = d.nxtA[v]; anc[v] = d.nxtB[v]; }
        }
        __threadfence_block();
        __syncthreads();
        const int a2 = any;
        __syncthreads();
        if (!a2) break;
    }
    // children lists: counts, exclusive scan, fill, sort each short list
    for (int v = threadIdx.x; v < n; v += kFinWG)
        if (par[v] >= 0) atomicAdd(&cnt[par[v] + 1], 1);
    __threadfence_block();
    __syncthreads();
    {
        const int t = threadIdx.x;
        const int chunk = (n + kFinWG - 1) / kFinWG;
        const int b = 1 + min(n, t * chunk), e = 1 + min(n, t * chunk + chunk);
        int loc = 0;
        for (int k = b; k < e; ++k) loc += cnt[k];
        sh[t] = loc;
        __syncthreads();
        for (int o = 1; o < kFinWG; o <<= 1) {
            const int add = (t >= o) ? sh[t - o] : 0;
            __syncthreads();
            sh[t] += add;
            __syncthreads();
        }
        int run = sh[t] - loc;
        __syncthreads();
        for (int k = b; k < e; ++k) { run += cnt[k]; cnt[k] = run; }
    }
    __threadfence_block();
    __syncthreads();
    for (int v = threadIdx.x; v <= n; v += kFinWG) d.child_off[v] = cnt[v];
    for (int v = threadIdx.x; v < n; v += kFinWG) anc[v] = cnt[v];   // fill cursors
    __threadfence_block();
    __syncthreads();
    for (int v = threadIdx.x; v < n; v += kFinWG)
        if (par[v] >= 0) d.child_idx[atomicAdd(&anc[par[v]], 1)] = v;
    __threadfence_block();
    __syncthreads();
    for (int v = threadIdx.x; v < n; v += kFinWG) {
        const int b = cnt[v], e = cnt[v + 1];
        int *ci = d.child_idx;
        if (e - b <= 8) {   // odd-even transposition sort of 8 register slots
            int r[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) r[k] = (b + k < e) ? ci[b + k] : 0x7fffffff;
#pragma unroll
            for (int pass = 0; pass < 8; ++pass) {
#pragma unroll
                for (int k = pass & 1; k + 1 < 8; k += 2) {
                    const int lo = min(r[k], r[k + 1]), hi = max(r[k], r[k + 1]);
                    r[k] = lo;
                    r[k + 1] = hi;
                }
            }
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (b + k < e) ci[b + k] = r[k];
        } else {
            for (int k = b + 1; k < e; ++k) {
                const int x = ci[k];
                int q = k - 1;
                while (q >= b && ci[q] > x) { ci[q + 1] = ci[q]; --q; }
                ci[q + 1] = x;
            }
        }
        if (LDS) {
            d.parent_new[v] = par[v];
            d.level_new[v] = lev[v];
        }
    }
}

void launch_mst_init(const Dev &d, hipStream_t s, const d4 *pos, int root_in) {
    k_mst_init<<<1, kTreeWG, 0, s>>>(d, pos, root_in);
}

// Dynamic LDS limit of the single-workgroup tree kernels, raised once per
// device to the largest size their launches request (150 KiB), so that
// launches themselves make no other runtime call (they may be captured).
static void tree_lds_limits() {
    static bool done[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64 || done[dev]) return;
    (void)hipFuncSetAttribute((const void *)k_bor_merge<true>, hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    (void)hipFuncSetAttribute((const void *)k_mst_finish<true>, hipFuncAttributeMaxDynamicSharedMemorySize, 150 * 1024);
    done[dev] = true;
}

void prepare_tree_launches() { tree_lds_limits(); }

// `rounds` Boruvka rounds (each a no-op once one component is left).
void launch_mst_rounds(const Dev &d, hipStream_t s, const d4 *pos, int rounds, int nsplit) {
    const int jchunk = (d.n + nsplit - 1) / nsplit;
    for (int r = 0; r < rounds; ++r) {
        k_bor_scan<<<dim3(d.nib, nsplit), 256, 0, s>>>(d, pos, jchunk);
        k_bor_vreduce<<<(d.n + kWG / 4 - 1) / (kWG / 4), kWG, 0, s>>>(d, nsplit);
        const size_t lds = (sizeof(unsigned long long) + 4 * sizeof(int)) * (size_t)d.n;
        if (lds <= 150 * 1024) {
            tree_lds_limits();
            k_bor_merge<true><<<1, kTreeWG, lds, s>>>(d);
        } else {
            k_bor_merge<false><<<1, kTreeWG, 0, s>>>(d);
        }
    }
}

void launch_mst_root(const Dev &d, hipStream_t s) {
    const size_t lds = sizeof(int) * (4 * (size_t)d.n + 1);
    if (lds <= 150 * 1024 && d.n <= 16 * kFinWG) {
        tree_lds_limits();
        k_mst_finish<true><<<1, kFinWG, lds, s>>>(d);
    } else {
        k_mst_finish<false><<<1, kFinWG, 0, s>>>(d);
    }
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
    if (u >= n || d.ctl->tree_bad) return;
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
    if (u >= n || d.ctl->tree_bad) return;
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
