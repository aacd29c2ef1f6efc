// Divide-and-conquer spanning tree on the GPU (paper Sec. 3.3).
//
// The bodies are grouped by an octree into about sqrt(N) parts; the tree is
// the union of every part's minimum spanning tree and of the minimum spanning
// tree of the meta-graph (one vertex per part, the edge between two parts
// weighing as their lightest connecting edge).  Every tree involved is the
// unique minimum spanning tree under the strict edge order (w, min index, max
// index) of the exact builder, so any correct algorithm yields the same edges:
//  * k_dc_keys:   bounding cube, cell coordinates at depth kDcDepth, Morton keys;
//  * k_dc_sort:   stable radix sort of (key, index), one workgroup;
//  * k_dc_octree: top-down split of every cell holding more than mcap bodies
//                 (not below depth kDcDepth); unsplit non-empty cells are the
//                 parts, numbered in key (depth-first octant) order;
//  * k_dc_local:  Prim inside each part, one wave per part (part in LDS);
//    each part becomes one component of the exact builder's Boruvka rounds,
//    its representative and tree root the part's first body.
// The rounds that follow (kernels_tree.hip) contract the components by their
// lightest outgoing edges: each component's lightest outgoing edge is its
// lightest meta-graph edge, so they are Boruvka's algorithm on the meta-graph
// and add exactly the edges of its minimum spanning tree, with the hooking
// component re-rooted at its end of the edge as for the exact tree.
#include "common.h"

namespace mstar {

namespace {

constexpr int kDcDepth = 10;     // finest octree depth (cell coordinates of 10 bits per axis)
constexpr int kDcWG = 1024;

__device__ __forceinline__ double dc_w(const d4 &a, const d4 &b) {
    const double dx = b.x - a.x, dy = b.y - a.y, dz = b.z - a.z;
    return (dx * dx + dy * dy) + dz * dz;   // the exact builder's weight, no contraction
}

// strict order (w, lo, hi)
__device__ __forceinline__ bool dc_less(double w1, int lo1, int hi1, double w2, int lo2, int hi2) {
    if (w1 < w2) return true;
    if (w1 > w2) return false;
    if (lo1 != lo2) return lo1 < lo2;
    return hi1 < hi2;
}

// Wave argmin of (w, lo, hi) with a payload; every lane ends with the minimum.
__device__ __forceinline__ void dc_wave_min(double &w, int &lo, int &hi, int &pay) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double w2 = __shfl_xor(w, off, 64);
        const int lo2 = __shfl_xor(lo, off, 64), hi2 = __shfl_xor(hi, off, 64), p2 = __shfl_xor(pay, off, 64);
        if (dc_less(w2, lo2, hi2, w, lo, hi)) { w = w2; lo = lo2; hi = hi2; pay = p2; }
    }
}

__device__ __forceinline__ unsigned spread3(unsigned v) {   // 10 bits -> every third bit
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

// Block reduction of min and max (thread 0's slots hold the results).
__device__ __forceinline__ void dc_minmax(double &lo, double &hi, double *s) {
    s[threadIdx.x] = lo;
    s[kDcWG + threadIdx.x] = hi;
    __syncthreads();
    for (int k = kDcWG / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) {
            s[threadIdx.x] = fmin(s[threadIdx.x], s[threadIdx.x + k]);
            s[kDcWG + threadIdx.x] = fmax(s[kDcWG + threadIdx.x], s[kDcWG + threadIdx.x + k]);
        }
        __syncthreads();
    }
    lo = s[0];
    hi = s[kDcWG];
    __syncthreads();
}

// Bounding cube, cell coordinates, Morton keys (x bit highest in each octant digit).
__global__ __launch_bounds__(kDcWG) void k_dc_keys(int n, const d4 *pos, DcBuf b) {
    __shared__ double s[2 * kDcWG];
    double lo[3], hi[3];
    for (int c = 0; c < 3; ++c) { lo[c] = INFINITY; hi[c] = -INFINITY; }
    for (int i = threadIdx.x; i < n; i += kDcWG) {
        const d4 p = pos[i];
        lo[0] = fmin(lo[0], p.x); hi[0] = fmax(hi[0], p.x);
        lo[1] = fmin(lo[1], p.y); hi[1] = fmax(hi[1], p.y);
        lo[2] = fmin(lo[2], p.z); hi[2] = fmax(hi[2], p.z);
    }
    for (int c = 0; c < 3; ++c) dc_minmax(lo[c], hi[c], s);
    double side = 0.0;
    for (int c = 0; c < 3; ++c) side = (hi[c] - lo[c] > side) ? hi[c] - lo[c] : side;
    constexpr int top = (1 << kDcDepth) - 1;
    const double inv = side > 0.0 ? (double)(1 << kDcDepth) / side : 0.0;
    for (int i = threadIdx.x; i < n; i += kDcWG) {
        const d4 p = pos[i];
        int k0 = (int)((p.x - lo[0]) * inv), k1 = (int)((p.y - lo[1]) * inv), k2 = (int)((p.z - lo[2]) * inv);
        k0 = k0 > top ? top : k0;
        k1 = k1 > top ? top : k1;
        k2 = k2 > top ? top : k2;
        b.key[i] = (spread3((unsigned)k0) << 2) | (spread3((unsigned)k1) << 1) | spread3((unsigned)k2);
        b.idx[i] = i;
    }
}

// Stable LSD radix sort of (key, idx) by 4-bit digits, 8 passes (the result
// returns to the first buffers).  Thread t owns a contiguous chunk of
// elements, counts its digits into its own column and scatters in order.
__global__ __launch_bounds__(kDcWG) void k_dc_sort(int n, DcBuf b) {
    __shared__ int cnt[16 * kDcWG];
    __shared__ int tot[kDcWG];
    const int t = threadIdx.x;
    const int chunk = (n + kDcWG - 1) / kDcWG;
    const int e0 = min(n, t * chunk), e1 = min(n, e0 + chunk);
    uint32_t *ks = b.key, *kd = b.key + n;
    int32_t *is = b.idx, *id = b.idx + n;
    for (int pass = 0; pass < 8; ++pass) {
        const int sh = 4 * pass;
        for (int d = 0; d < 16; ++d) cnt[d * kDcWG + t] = 0;
        for (int e = e0; e < e1; ++e) cnt[((ks[e] >> sh) & 15u) * kDcWG + t] += 1;
        __syncthreads();
        // exclusive scan of cnt[] in digit-major order: thread t owns entries [16 t, 16 t + 16)
        int loc[16], s = 0;
        for (int k = 0; k < 16; ++k) { loc[k] = s; s += cnt[16 * t + k]; }
        tot[t] = s;
        __syncthreads();
        for (int off = 1; off < kDcWG; off <<= 1) {   // inclusive scan of the totals
            const int v = t >= off ? tot[t - off] : 0;
            __syncthreads();
            tot[t] += v;
            __syncthreads();
        }
        const int base = tot[t] - s;
        for (int k = 0; k < 16; ++k) cnt[16 * t + k] = base + loc[k];
        __syncthreads();
        for (int e = e0; e < e1; ++e) {
            const uint32_t k = ks[e];
            const int slot = ((k >> sh) & 15u) * kDcWG + t;
            const int dst = cnt[slot];
            cnt[slot] = dst + 1;
            kd[dst] = k;
            id[dst] = is[e];
        }
        __threadfence_block();
        __syncthreads();
        uint32_t *tk = ks; ks = kd; kd = tk;
        int32_t *ti = is; is = id; id = ti;
    }
}

// Top-down octree on the sorted keys; leaves (parts) marked at their first
// sorted position, then numbered by a scan.  Also the part of every body,
// the part ranges and the sorted positions.
__global__ __launch_bounds__(kDcWG) void k_dc_octree(Dev d, int mcap, const d4 *pos, DcBuf b) {
    const int n = d.n;
    __shared__ int na, nb2;
    __shared__ int tot[kDcWG];
    const int t = threadIdx.x;
    for (int i = t; i <= n; i += kDcWG) b.flag[i] = 0;
    if (t == 0) {
        b.cells[0] = make_int2(0, n);
        na = 1;
    }
    __threadfence_block();
    __syncthreads();
    int2 *A = b.cells, *B = b.cells + n;
    for (int level = 0; level <= kDcDepth; ++level) {
        if (t == 0) nb2 = 0;
        __syncthreads();
        const int cnt = na;
        for (int c = t; c < cnt; c += kDcWG) {
            const int2 r = A[c];
            if (r.y - r.x > mcap && level < kDcDepth) {
                const int sh = 3 * (kDcDepth - 1 - level);
                int start = r.x;
                for (int dig = 0; dig < 8; ++dig) {
                    // first position in [start, r.y) whose digit exceeds dig
                    int lo = start, hi = r.y;
                    while (lo < hi) {
                        const int mid = (lo + hi) >> 1;
                        if ((int)((b.key[mid] >> sh) & 7u) <= dig) lo = mid + 1;
                        else hi = mid;
                    }
                    if (lo > start) B[atomicAdd(&nb2, 1)] = make_int2(start, lo);
                    start = lo;
                }
            } else {
                b.flag[r.x] = 1;
            }
        }
        __threadfence_block();
        __syncthreads();
        if (t == 0) na = nb2;
        __syncthreads();
        int2 *tmp = A; A = B; B = tmp;
        if (na == 0) break;
    }
    // part numbers: inclusive scan of the leaf flags over sorted positions
    const int chunk = (n + kDcWG - 1) / kDcWG;
    const int e0 = min(n, t * chunk), e1 = min(n, e0 + chunk);
    int s = 0;
    for (int e = e0; e < e1; ++e) s += b.flag[e];
    tot[t] = s;
    __syncthreads();
    for (int off = 1; off < kDcWG; off <<= 1) {
        const int v = t >= off ? tot[t - off] : 0;
        __syncthreads();
        tot[t] += v;
        __syncthreads();
    }
    int run = tot[t] - s;
    const int np = tot[kDcWG - 1];
    for (int e = e0; e < e1; ++e) {
        if (b.flag[e]) {
            b.pstart[run] = e;
            ++run;
        }
        const int p = run - 1;
        const int body = b.idx[e];
        b.part[body] = p;
        b.spos[e] = pos[body];
    }
    if (t == 0) {   // the parts are the components the Boruvka rounds start from
        *b.np = np;
        b.pstart[np] = n;
        *d.ncomp = np;
        *d.done = np <= 1 ? 1 : 0;
    }
}

// Prim inside each part (one wave per part, parts strided over the grid).
// A part of at most kLocalMax bodies is held in LDS; a larger one (possible
// only for a cell at the finest depth) keeps its tree state per sorted
// position in global memory, each position read and written only by the lane
// that owns it (k - s0 - 1 mod 64).  Every body is labelled with its part's
// component, the part's first body, which is also the part tree's root.
constexpr int kLocalMax = 512;

__global__ __launch_bounds__(64) void k_dc_local(Dev d, DcBuf b) {
    __shared__ double sx[kLocalMax], sy[kLocalMax], sz[kLocalMax], sw[kLocalMax];
    __shared__ int su[kLocalMax], sv[kLocalMax], sf[kLocalMax];
    const int np = *b.np;
    const int lane = threadIdx.x;
    for (int p = blockIdx.x; p < np; p += gridDim.x) {
        const int s0 = b.pstart[p], s1 = b.pstart[p + 1], cnt = s1 - s0;
        const int r = b.idx[s0];
        for (int k = s0 + lane; k < s1; k += 64) d.comp[b.idx[k]] = r;
        if (lane == 0) d.parent_new[r] = -1;
        if (cnt <= kLocalMax) {
            __syncthreads();   // the previous part's LDS reads are done
            for (int k = lane; k < cnt; k += 64) {
                const d4 q = b.spos[s0 + k];
                sx[k] = q.x; sy[k] = q.y; sz[k] = q.z;
                sv[k] = b.idx[s0 + k];
                sf[k] = 0;
            }
            __syncthreads();
            const d4 q0{sx[0], sy[0], sz[0], 0.0};
            for (int k = 1 + lane; k < cnt; k += 64) {
                sw[k] = dc_w(q0, d4{sx[k], sy[k], sz[k], 0.0});
                su[k] = r;
            }
            __syncthreads();
            for (int step = 1; step < cnt; ++step) {
                double w = INFINITY;
                int lo = 0x7fffffff, hi = 0x7fffffff, pay = -1;
                for (int k = 1 + lane; k < cnt; k += 64) {
                    if (sf[k]) continue;
                    const int u = su[k], v = sv[k];
                    const int l2 = min(u, v), h2 = max(u, v);
                    if (pay < 0 || dc_less(sw[k], l2, h2, w, lo, hi)) { w = sw[k]; lo = l2; hi = h2; pay = k; }
                }
                dc_wave_min(w, lo, hi, pay);
                const int pick = pay;
                const int vb = sv[pick];
                const d4 pp{sx[pick], sy[pick], sz[pick], 0.0};
                if (((pick - 1) & 63) == lane) {   // the lane that owns the picked slot
                    sf[pick] = 1;
                    d.parent_new[vb] = su[pick];
                }
                for (int k = 1 + lane; k < cnt; k += 64) {
                    if (sf[k]) continue;
                    const double wk = dc_w(pp, d4{sx[k], sy[k], sz[k], 0.0});
                    const int v = sv[k];
                    if (dc_less(wk, min(vb, v), max(vb, v), sw[k], min(su[k], v), max(su[k], v))) {
                        sw[k] = wk;
                        su[k] = vb;
                    }
                }
            }
            continue;
        }
        {
            const d4 pr = b.spos[s0];
            for (int k = s0 + 1 + lane; k < s1; k += 64) {
                b.bw[k] = dc_w(pr, b.spos[k]);
                b.bu[k] = r;
                b.in[k] = 0;
            }
        }
        for (int step = s0 + 1; step < s1; ++step) {
            double w = INFINITY;
            int lo = 0x7fffffff, hi = 0x7fffffff, pay = -1;
            for (int k = s0 + 1 + lane; k < s1; k += 64) {
                if (b.in[k]) continue;
                const int u = b.bu[k], v = b.idx[k];
                const int l2 = min(u, v), h2 = max(u, v);
                if (pay < 0 || dc_less(b.bw[k], l2, h2, w, lo, hi)) { w = b.bw[k]; lo = l2; hi = h2; pay = k; }
            }
            dc_wave_min(w, lo, hi, pay);
            const int pick = pay;
            const int vb = b.idx[pick];
            const d4 pp = b.spos[pick];
            if (((pick - s0 - 1) & 63) == lane) {
                b.in[pick] = 1;
                d.parent_new[vb] = b.bu[pick];
            }
            for (int k = s0 + 1 + lane; k < s1; k += 64) {
                if (b.in[k]) continue;
                const double wk = dc_w(pp, b.spos[k]);
                const int v = b.idx[k];
                if (dc_less(wk, min(vb, v), max(vb, v), b.bw[k], min(b.bu[k], v), max(b.bu[k], v))) {
                    b.bw[k] = wk;
                    b.bu[k] = vb;
                }
            }
        }
    }
}

}  // namespace

void launch_mst_dc(const Dev &d, const DcBuf &b, hipStream_t s, const d4 *pos, int mcap) {
    k_dc_keys<<<1, kDcWG, 0, s>>>(d.n, pos, b);
    k_dc_sort<<<1, kDcWG, 0, s>>>(d.n, b);
    k_dc_octree<<<1, kDcWG, 0, s>>>(d, mcap, pos, b);
    k_dc_local<<<std::min(d.n, 2048), 64, 0, s>>>(d, b);
}

}  // namespace mstar
