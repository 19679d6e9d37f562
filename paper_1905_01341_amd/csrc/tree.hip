// Octree construction on the GPU (Section 3.9: cube scaling, level-wise
// subdivision, empty boxes skipped, bit interleaving + sort, neighbour and
// interaction lists, built once per mesh).
//
// Steps: bounding cube -> 45-bit Morton keys (15 bits per axis) -> stable
// LSD radix sort of (key, point) in six 8-bit passes -> per-level unique
// prefixes (boxes) by flag + scan -> parent / child / neighbour tables by
// binary search in the sorted per-level key arrays -> M2L pairs (children
// of the parent's neighbours that are not adjacent) and M2M/L2L pairs,
// grouped by translation operator.
#include <algorithm>
#include <climits>
#include <cmath>

#include "common.h"
#include "ops.h"
#include "tree.h"
#include "xcd.h"

namespace bfm {

static unsigned nblk(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// fill with a value (a kernel rather than a memset, so that the same code can
// be replayed from a captured graph)
__global__ void k_fill_int(int *p, int64_t n, int v) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
__global__ void k_fill_u64(unsigned long long *p, int64_t n, unsigned long long v) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}


// ---------------------------------------------------------------------------
// Morton keys

__host__ __device__ inline uint64_t spread3(uint32_t v) {
    uint64_t x = v & 0x1fffffu;  // up to 21 bits
    x = (x | (x << 32)) & 0x1f00000000ffffull;
    x = (x | (x << 16)) & 0x1f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__host__ __device__ inline uint32_t compact3(uint64_t x) {
    x &= 0x1249249249249249ull;
    x = (x ^ (x >> 2)) & 0x10c30c30c30c30c3ull;
    x = (x ^ (x >> 4)) & 0x100f00f00f00f00full;
    x = (x ^ (x >> 8)) & 0x1f0000ff0000ffull;
    x = (x ^ (x >> 16)) & 0x1f00000000ffffull;
    x = (x ^ (x >> 32)) & 0x1fffffull;
    return (uint32_t)x;
}

// key = ... x_b y_b z_b ... (x in the highest bit of every triple)
__host__ __device__ inline uint64_t morton(uint32_t ix, uint32_t iy, uint32_t iz) {
    return (spread3(ix) << 2) | (spread3(iy) << 1) | spread3(iz);
}

__host__ __device__ inline void demorton(uint64_t k, int &ix, int &iy, int &iz) {
    ix = (int)compact3(k >> 2);
    iy = (int)compact3(k >> 1);
    iz = (int)compact3(k);
}

// ---------------------------------------------------------------------------
// Bounding box

__global__ void k_bbox_partial(const double *xyz, int64_t n, double *part) {
    __shared__ double smin[3][256], smax[3][256];
    double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        for (int d = 0; d < 3; ++d) {
            double v = xyz[3 * i + d];
            mn[d] = fmin(mn[d], v);
            mx[d] = fmax(mx[d], v);
        }
    }
    for (int d = 0; d < 3; ++d) {
        smin[d][threadIdx.x] = mn[d];
        smax[d][threadIdx.x] = mx[d];
    }
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int d = 0; d < 3; ++d) {
                smin[d][threadIdx.x] = fmin(smin[d][threadIdx.x], smin[d][threadIdx.x + s]);
                smax[d][threadIdx.x] = fmax(smax[d][threadIdx.x], smax[d][threadIdx.x + s]);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int d = 0; d < 3; ++d) {
            part[6 * blockIdx.x + d] = smin[d][0];
            part[6 * blockIdx.x + 3 + d] = smax[d][0];
        }
}

// The cube from the partial boxes, on the device (the Morton pass reads it
// without a wait for the host): geo = (origin x, y, z, side, 2^kKeyBits /
// side, all bounds finite ? 1 : 0). The cube is the box's largest extent
// enlarged by 1e-9 relative, centred on the box.
__global__ void __launch_bounds__(256) k_bbox_final(const double *part, int nbb, double *geo) {
    __shared__ double smin[3][256], smax[3][256];
    double mn[3] = {1e300, 1e300, 1e300}, mx[3] = {-1e300, -1e300, -1e300};
    for (int b = threadIdx.x; b < nbb; b += 256)
        for (int d = 0; d < 3; ++d) {
            mn[d] = fmin(mn[d], part[6 * b + d]);
            mx[d] = fmax(mx[d], part[6 * b + 3 + d]);
        }
    for (int d = 0; d < 3; ++d) {
        smin[d][threadIdx.x] = mn[d];
        smax[d][threadIdx.x] = mx[d];
    }
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int d = 0; d < 3; ++d) {
                smin[d][threadIdx.x] = fmin(smin[d][threadIdx.x], smin[d][threadIdx.x + s]);
                smax[d][threadIdx.x] = fmax(smax[d][threadIdx.x], smax[d][threadIdx.x + s]);
            }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        double ext = 0.0;
        bool fin = true;
        for (int d = 0; d < 3; ++d) {
            fin = fin && isfinite(smin[d][0]) && isfinite(smax[d][0]);
            ext = fmax(ext, smax[d][0] - smin[d][0]);
        }
        if (!(ext > 0.0)) ext = 1.0;
        const double side = ext * (1.0 + 1e-9) + 1e-300;
        for (int d = 0; d < 3; ++d) geo[d] = 0.5 * (smin[d][0] + smax[d][0]) - 0.5 * side;
        geo[3] = side;
        geo[4] = (double)(1 << kKeyBits) / side;
        geo[5] = fin ? 1.0 : 0.0;
    }
}

__global__ void k_morton(const double *xyz, int64_t n, const double *geo, uint64_t *key, int *idx) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int lim = (1 << kKeyBits) - 1;
    int c[3];
    const double o[3] = {geo[0], geo[1], geo[2]};
    const double inv_cell = geo[4];
    for (int d = 0; d < 3; ++d) {
        double f = floor((xyz[3 * i + d] - o[d]) * inv_cell);
        int v = (int)fmin(fmax(f, 0.0), (double)lim);
        c[d] = v;
    }
    key[i] = morton(c[0], c[1], c[2]);
    idx[i] = (int)i;
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort of (uint64 key, int value), 8 bits per pass.
// Tiles of 4096 items per 256-thread block; each wave ranks its 1024-item
// segment in order with ballot-based digit matching, so equal digits keep
// their input order (stability).

constexpr int RS_THREADS = 256;
constexpr int RS_TILE = 4096;
constexpr int RS_SEG = 1024;  // per wave
constexpr int RS_ROUNDS = RS_SEG / 64;

__global__ void __launch_bounds__(RS_THREADS) k_rs_hist(const uint64_t *keys, int64_t n, int shift,
                                                        int *hist, int nblocks) {
    __shared__ int cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * RS_TILE;
    for (int k = 0; k < RS_TILE / RS_THREADS; ++k) {
        int64_t i = base + k * RS_THREADS + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 255], 1);
    }
    __syncthreads();
    hist[threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

__global__ void __launch_bounds__(RS_THREADS) k_rs_scatter(const uint64_t *kin, const int *vin,
                                                           int64_t n, int shift, const int *scanned,
                                                           int nblocks, uint64_t *kout, int *vout) {
    __shared__ int wcnt[4][256];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int d = threadIdx.x; d < 4 * 256; d += RS_THREADS) (&wcnt[0][0])[d] = 0;
    __syncthreads();
    const int64_t seg = (int64_t)blockIdx.x * RS_TILE + (int64_t)w * RS_SEG;
    uint64_t kreg[RS_ROUNDS];
    int vreg[RS_ROUNDS], pos[RS_ROUNDS];
    const uint64_t lt = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    for (int r = 0; r < RS_ROUNDS; ++r) {
        const int64_t i = seg + r * 64 + lane;
        const bool ok = i < n;
        kreg[r] = ok ? kin[i] : 0;
        vreg[r] = ok ? vin[i] : 0;
        const int d = ok ? (int)((kreg[r] >> shift) & 255) : 256;
        uint64_t peers = __ballot(ok);
        for (int b = 0; b < 8; ++b) {
            uint64_t bal = __ballot(ok && ((d >> b) & 1));
            peers &= ((d >> b) & 1) ? bal : ~bal;
        }
        int base = 0;
        if (ok) base = wcnt[w][d];
        __builtin_amdgcn_wave_barrier();
        const int rank = __popcll(peers & lt);
        pos[r] = base + rank;
        if (ok && rank == 0) wcnt[w][d] = base + __popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    {  // exclusive prefix over the 4 waves for digit d = threadIdx.x
        const int d = threadIdx.x;
        int run = 0;
        for (int ww = 0; ww < 4; ++ww) {
            int t = wcnt[ww][d];
            wcnt[ww][d] = run + scanned[d * nblocks + blockIdx.x];
            run += t;
        }
    }
    __syncthreads();
    for (int r = 0; r < RS_ROUNDS; ++r) {
        const int64_t i = seg + r * 64 + lane;
        if (i < n) {
            const int d = (int)((kreg[r] >> shift) & 255);
            const int p = wcnt[w][d] + pos[r];
            kout[p] = kreg[r];
            vout[p] = vreg[r];
        }
    }
}

// Stable LSD sort of (keys, vals) by key bits [lo, lo + bits), 8 bits a pass.
static void radix_sort_range(uint64_t *keys, int *vals, uint64_t *keys_tmp, int *vals_tmp, int64_t n, int lo,
                             int bits, Tree::Scratch &scr, hipStream_t st) {
    if (n <= 1) return;
    const int nblocks = (int)((n + RS_TILE - 1) / RS_TILE);
    DevBuf<int> &hist = scr.rs_hist, &scanned = scr.rs_scanned, &tmp = scr.rs_tmp;
    hist.ensure((size_t)256 * nblocks);
    scanned.ensure((size_t)256 * nblocks);
    uint64_t *kin = keys, *kout = keys_tmp;
    int *vin = vals, *vout = vals_tmp;
    int passes = (bits + 7) / 8;
    if (passes & 1) ++passes;  // even pass count: the result lands back in keys / vals
    for (int pass = 0; pass < passes; ++pass) {
        const int shift = lo + 8 * pass;
        k_rs_hist<<<nblocks, RS_THREADS, 0, st>>>(kin, n, shift, hist.get(), nblocks);
        BFM_LAUNCHED();
        exclusive_scan_async(hist.get(), scanned.get(), (int64_t)256 * nblocks, st, tmp);
        k_rs_scatter<<<nblocks, RS_THREADS, 0, st>>>(kin, vin, n, shift, scanned.get(), nblocks, kout, vout);
        BFM_LAUNCHED();
        std::swap(kin, kout);
        std::swap(vin, vout);
    }
}

void radix_sort(uint64_t *keys, int *vals, uint64_t *keys_tmp, int *vals_tmp, int64_t n, int bits, Tree::Scratch &scr,
                hipStream_t st) {
    radix_sort_range(keys, vals, keys_tmp, vals_tmp, n, 0, bits, scr, st);
}

// ---------------------------------------------------------------------------
// Exclusive scan (int32)

constexpr int SC_THREADS = 1024;
constexpr int SC_TILE = 4096;

__global__ void __launch_bounds__(SC_THREADS) k_scan_tile(const int *in, int *out, int64_t n,
                                                          int *sums) {
    __shared__ int ts[SC_THREADS];
    const int64_t base = (int64_t)blockIdx.x * SC_TILE + threadIdx.x * 4;
    int v[4], s = 0;
    for (int k = 0; k < 4; ++k) {
        v[k] = (base + k < n) ? in[base + k] : 0;
        s += v[k];
    }
    ts[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < SC_THREADS; off <<= 1) {
        int t = (threadIdx.x >= (unsigned)off) ? ts[threadIdx.x - off] : 0;
        __syncthreads();
        ts[threadIdx.x] += t;
        __syncthreads();
    }
    int run = ts[threadIdx.x] - s;  // exclusive prefix of this thread
    for (int k = 0; k < 4; ++k) {
        if (base + k < n) out[base + k] = run;
        run += v[k];
    }
    if (threadIdx.x == SC_THREADS - 1 && sums) sums[blockIdx.x] = ts[SC_THREADS - 1];
}

__global__ void k_scan_add(int *out, int64_t n, const int *offs) {
    int64_t i = (int64_t)blockIdx.x * SC_TILE + threadIdx.x;
    const int o = offs[blockIdx.x];
    for (int k = 0; k < SC_TILE; k += blockDim.x)
        if (i + k < n && i + k < (int64_t)(blockIdx.x + 1) * SC_TILE) out[i + k] += o;
}

static void scan_rec(const int *in, int *out, int64_t n, hipStream_t st, int *tmp) {
    const int64_t nb = (n + SC_TILE - 1) / SC_TILE;
    if (nb <= 1) {
        k_scan_tile<<<1, SC_THREADS, 0, st>>>(in, out, n, nullptr);
        BFM_LAUNCHED();
        return;
    }
    int *sums = tmp;
    k_scan_tile<<<(unsigned)nb, SC_THREADS, 0, st>>>(in, out, n, sums);
    BFM_LAUNCHED();
    scan_rec(sums, sums, nb, st, tmp + nb);
    k_scan_add<<<(unsigned)nb, 256, 0, st>>>(out, n, sums);
    BFM_LAUNCHED();
}

// total = in[n-1] (kept before an in-place scan overwrites it), then
// total += out[n-1]: the sum of all inputs, on the device
__global__ void k_scan_last(const int *in, int64_t n, int *total) {
    if (threadIdx.x == 0 && blockIdx.x == 0) total[0] = in[n - 1];
}
__global__ void k_scan_total(const int *out, int64_t n, int *total) {
    if (threadIdx.x == 0 && blockIdx.x == 0) total[0] += out[n - 1];
}

// totals of three exclusive scans of n >= 1 counts: last offset + last count
__global__ void k_scan_totals3(const int *c0, const int *o0, const int *c1, const int *o1, const int *c2,
                               const int *o2, int64_t n, int *out) {
    if (threadIdx.x == 0) {
        out[0] = o0[n - 1] + c0[n - 1];
        out[1] = o1[n - 1] + c1[n - 1];
        out[2] = o2[n - 1] + c2[n - 1];
    }
}

// scratch of the recursion (the sums of every level) plus one slot for the
// total at index *total_slot
static int *scan_scratch(int64_t n, DevBuf<int> &tmp, int64_t *total_slot = nullptr) {
    int64_t need = 2, m = n;
    while (m > 1) {
        m = (m + SC_TILE - 1) / SC_TILE;
        need += m + 1;
    }
    if (total_slot) *total_slot = need + 1;
    return tmp.ensure((size_t)need + 2);
}

void exclusive_scan_async(const int *in, int *out, int64_t n, hipStream_t st, DevBuf<int> &tmp) {
    if (n <= 0) return;
    scan_rec(in, out, n, st, scan_scratch(n, tmp));
}

// ---------------------------------------------------------------------------
// Levels

__global__ void k_level_counts(const uint64_t *key, int64_t n, int lmax, unsigned long long *counts) {
    __shared__ int c[kKeyBits + 1];
    if (threadIdx.x <= kKeyBits) c[threadIdx.x] = 0;
    __syncthreads();
    // a grid of a few hundred workgroups strides over the points, so that the
    // global counters take few adds; within a workgroup one LDS add per wave
    // and level (at the deep levels nearly every point opens a box)
    for (int64_t i0 = blockIdx.x * (int64_t)blockDim.x; i0 < n; i0 += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = i0 + threadIdx.x;
        const uint64_t ki = i < n ? key[i] : 0, kp = (i > 0 && i < n) ? key[i - 1] : 0;
        for (int l = 0; l <= lmax; ++l) {
            const int sh = 3 * (kKeyBits - l);
            const uint64_t opens = __ballot(i < n && (i == 0 || (ki >> sh) != (kp >> sh)));
            if ((threadIdx.x & 63) == 0 && opens) atomicAdd(&c[l], (int)__popcll(opens));
        }
    }
    __syncthreads();
    if (threadIdx.x <= (unsigned)lmax && c[threadIdx.x])
        atomicAdd(&counts[threadIdx.x], (unsigned long long)c[threadIdx.x]);
}

// Boxes of every level 0..lmax in one pass. Entry e = l n + i flags point i
// when it opens a box of level l (its key differs from point i-1's at that
// level). Levels are numbered one after the other, so an exclusive scan over
// all (lmax + 1) n flags gives every box its global index directly.
__global__ void k_level_flags(const uint64_t *key, int64_t n, int lmax, int *flag) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)(lmax + 1) * n) return;
    const int l = (int)(e / n);
    const int64_t i = e - (int64_t)l * n;
    const int shift = 3 * (kKeyBits - l);
    flag[e] = (i == 0 || (key[i] >> shift) != (key[i - 1] >> shift)) ? 1 : 0;
}

// Box key, level and first point of every box; pt_leaf[i] = leaf (level
// lmax box, counted from leaf0) of point i.
__global__ void k_level_scatter(const uint64_t *key, int64_t n, int lmax, const int *flag, const int *pos,
                                int64_t leaf0, uint64_t *box_key, int *box_level, int *box_pt0, int *pt_leaf) {
    const int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (e >= (int64_t)(lmax + 1) * n) return;
    const int l = (int)(e / n);
    const int64_t i = e - (int64_t)l * n;
    if (l == lmax) pt_leaf[i] = (int)(pos[e] + flag[e] - 1 - leaf0);  // inclusive count - 1
    if (!flag[e]) return;
    const int64_t b = pos[e];
    box_key[b] = key[i] >> (3 * (kKeyBits - l));
    box_level[b] = l;
    box_pt0[b] = (int)i;
}

__device__ inline int64_t lower_bound_u64(const uint64_t *a, int64_t lo, int64_t hi, uint64_t v) {
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (a[mid] < v)
            lo = mid + 1;
        else
            hi = mid;
    }
    return lo;
}

struct LevelInfo {
    int64_t off[kKeyBits + 2];
    double h[kKeyBits + 1];
};

// One thread per (box, neighbour slot): the slot's neighbour by binary search
// in the box's level; the thread of slot 13 (the box itself) also writes the
// box's centre and parent.
__global__ void k_box_meta(int64_t nbox, int lmax, LevelInfo li, double ox, double oy, double oz,
                           const uint64_t *box_key, const int *box_level, int *box_parent, double *centre,
                           int *nbr) {
    const int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (g >= 27 * nbox) return;
    const int64_t b = g / 27;
    const int s = (int)(g - 27 * b);
    const int l = box_level[b];
    const uint64_t k = box_key[b];
    int ix, iy, iz;
    demorton(k, ix, iy, iz);
    if (s == 13) {
        const double h = li.h[l];
        centre[3 * b] = ox + (ix + 0.5) * h;
        centre[3 * b + 1] = oy + (iy + 0.5) * h;
        centre[3 * b + 2] = oz + (iz + 0.5) * h;
        box_parent[b] = (l == 0) ? -1 : (int)lower_bound_u64(box_key, li.off[l - 1], li.off[l], k >> 3);
    }
    const int lim = 1 << l;
    const int dx = s / 9 - 1, dy = (s / 3) % 3 - 1, dz = s % 3 - 1;
    const int jx = ix + dx, jy = iy + dy, jz = iz + dz;
    int res = -1;
    if (jx >= 0 && jy >= 0 && jz >= 0 && jx < lim && jy < lim && jz < lim) {
        const uint64_t nk = morton(jx, jy, jz);
        const int64_t q = lower_bound_u64(box_key, li.off[l], li.off[l + 1], nk);
        if (q < li.off[l + 1] && box_key[q] == nk) res = (int)q;
    }
    nbr[27 * b + s] = res;
    (void)lmax;
}

// Number of near-field pairs per leaf, and leaf point ranges.
__global__ void k_leaf_near(int64_t nleaf, int64_t leaf0, const int *box_pt0, int64_t npts,
                            const int *nbr, int *leaf_pt, unsigned long long *pairs, int *maxocc) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nleaf) return;
    const int64_t b = leaf0 + i;
    const int p0 = box_pt0[b];
    const int p1 = (i + 1 < nleaf) ? box_pt0[b + 1] : (int)npts;
    leaf_pt[i] = p0;
    if (i + 1 == nleaf) leaf_pt[nleaf] = (int)npts;
    unsigned long long src = 0;
    for (int s = 0; s < 27; ++s) {
        const int q = nbr[27 * b + s];
        if (q < 0) continue;
        const int64_t qi = q - leaf0;
        const int q0 = box_pt0[q];
        const int q1 = (qi + 1 < nleaf) ? box_pt0[q + 1] : (int)npts;
        src += (unsigned long long)(q1 - q0);
    }
    atomicAdd(pairs, src * (unsigned long long)(p1 - p0));
    atomicMax(maxocc, p1 - p0);
}

// Merged near-field source ranges per leaf: the existing neighbours' point
// ranges sorted by start, touching ranges joined (Morton order makes many
// neighbours adjacent in the sorted point array).
__global__ void __launch_bounds__(256) k_leaf_ranges(int64_t nleaf, int64_t leaf0, const int *leaf_pt,
                                                     const int *nbr, int2 *rng, int *cnt) {
    // one wave per leaf: lane s < 27 holds neighbour slot s's point range;
    // the ranges are ranked by start, and contiguous ones merged
    __shared__ int2 sorted[4][32];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6;
    if (i >= nleaf) return;  // the whole wave
    const int64_t b = leaf0 + i;
    int a = INT_MAX, e = 0;
    const int q = lane < 27 ? nbr[27 * b + lane] : -1;
    if (q >= 0) {
        a = leaf_pt[q - leaf0];
        e = leaf_pt[q - leaf0 + 1];
    }
    int rank = 0;  // leaves are non-empty, so the starts are distinct
    for (int y = 0; y < 27; ++y) rank += __shfl(a, y) < a ? 1 : 0;
    const int k = __popcll(__ballot(q >= 0));
    if (q >= 0) sorted[w][rank] = make_int2(a, e);
    __builtin_amdgcn_wave_barrier();
    const int2 me = lane < k ? sorted[w][lane] : make_int2(0, 0);
    const int eprev = __shfl_up(me.y, 1);
    const bool start = lane < k && (lane == 0 || eprev != me.x);
    const uint64_t starts = __ballot(start);
    const bool last = lane < k && (lane == k - 1 || ((starts >> (lane + 1)) & 1ull));
    const int run = __popcll(starts & ((2ull << lane) - 1ull)) - 1;  // runs begun at lanes <= this one
    int *out = reinterpret_cast<int *>(rng + 27 * i);
    if (start) out[2 * run] = me.x;
    if (last) out[2 * run + 1] = me.y;
    if (lane == 0) cnt[i] = __popcll(starts);
}

// Leaf work items (P2M, L2P): chunks of at most kLeafChunk points per leaf.
__global__ void k_item_count(int64_t nleaf, const int *leaf_pt, int *cnt) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nleaf) return;
    cnt[i] = (leaf_pt[i + 1] - leaf_pt[i] + kLeafChunk - 1) / kLeafChunk;
}

__global__ void k_item_fill(int64_t nleaf, const int *leaf_pt, const int *off, int2 *items) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nleaf) return;
    const int r0 = leaf_pt[i], r1 = leaf_pt[i + 1];
    int o = off[i];
    for (int r = r0; r < r1; r += kLeafChunk, ++o) items[o] = make_int2((int)i, r);
}

// near-field sources of leaf i and the number of pieces they are split into
__device__ inline int leaf_sources(int64_t i, const int2 *rng, const int *rcnt) {
    int src = 0;
    for (int k = 0; k < rcnt[i]; ++k) src += rng[27 * i + k].y - rng[27 * i + k].x;
    return src;
}

__global__ void k_piece_count(int64_t nleaf, const int *leaf_pt, const int2 *rng, const int *rcnt, int *cnt,
                              int *split) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nleaf) return;
    const int src = leaf_sources(i, rng, rcnt);
    const int pieces = src > 0 ? (src + kP2PPiece - 1) / kP2PPiece : 1;
    cnt[i] = pieces * ((leaf_pt[i + 1] - leaf_pt[i] + kP2PChunk - 1) / kP2PChunk);
    if (pieces > 1) split[0] = 1;  // any writer stores the same value
}

__global__ void k_piece_fill(int64_t nleaf, const int *leaf_pt, const int *off, const int2 *rng, const int *rcnt,
                             int4 *items) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nleaf) return;
    const int src = leaf_sources(i, rng, rcnt);
    const int pieces = src > 0 ? (src + kP2PPiece - 1) / kP2PPiece : 1;
    const int ps = (src + pieces - 1) / pieces;  // balanced piece length
    const int r0 = leaf_pt[i], r1 = leaf_pt[i + 1];
    int o = off[i];
    for (int r = r0; r < r1; r += kP2PChunk)
        for (int p = 0; p < pieces; ++p, ++o) items[o] = make_int4((int)i, r, min(src, p * ps), min(src, (p + 1) * ps));
}

// Symmetric near-field items: chunk [r0, r1) (at most `chunk` receivers) of
// leaf i takes its near ranges clipped to start at r0; positions [0, r1 - r0)
// are the chunk itself (split into pieces of dpiece), the rest into pieces of
// `piece`.
__device__ inline int sym_list_len(int64_t i, int r0, const int2 *rng, const int *rcnt) {
    int len = 0;
    for (int k = 0; k < rcnt[i]; ++k) len += max(0, rng[27 * i + k].y - max(rng[27 * i + k].x, r0));
    return len;
}

template <bool FILL>
__global__ void k_sym_items(int64_t nleaf, const int *leaf_pt, const int2 *rng, const int *rcnt, SymShape sh,
                            int *cnt, const int *off, int4 *items) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= nleaf) return;
    const int p0 = leaf_pt[i], p1 = leaf_pt[i + 1];
    int o = FILL ? off[i] : 0;
    for (int r0 = p0; r0 < p1; r0 += sh.chunk) {
        const int d = min(r0 + sh.chunk, p1) - r0;
        const int len = sym_list_len(i, r0, rng, rcnt);
        for (int s = 0; s < d; s += sh.dpiece, ++o)
            if (FILL) items[o] = make_int4((int)i, r0, s, min(d, s + sh.dpiece));
        for (int s = d; s < len; s += sh.piece, ++o)
            if (FILL) items[o] = make_int4((int)i, r0, s, min(len, s + sh.piece));
    }
    if (!FILL) cnt[i] = o;
}

// ---------------------------------------------------------------------------
// Interaction lists

__constant__ signed short c_m2l_lut[343];

__device__ inline void child_range(const uint64_t *box_key, const LevelInfo &li, int l, uint64_t k,
                                   int64_t &c0, int64_t &c1) {
    c0 = lower_bound_u64(box_key, li.off[l + 1], li.off[l + 2], k << 3);
    c1 = lower_bound_u64(box_key, li.off[l + 1], li.off[l + 2], (k + 1) << 3);
}

__device__ inline void m2l_pairs_one(int mode, int64_t t, int64_t b0, const LevelInfo &li, const uint64_t *box_key,
                                     const int *box_level, const int *box_parent, const int *nbr, int *count,
                                     const int *offs, int *tsrc, int *tdst, int *top, int *lh) {
    const int64_t b = b0 + t / 27;
    const int s = (int)(t % 27);
    const int q = nbr[27 * (int64_t)box_parent[b] + s];
    int c = 0;
    if (q >= 0) {
        const int l = box_level[b];
        int ix, iy, iz;
        demorton(box_key[b], ix, iy, iz);
        int64_t w = (mode == 1) ? offs[t] : 0;
        int64_t c0, c1;
        child_range(box_key, li, l - 1, box_key[q], c0, c1);
        for (int64_t cc = c0; cc < c1; ++cc) {
            int jx, jy, jz;
            demorton(box_key[cc], jx, jy, jz);
            const int dx = ix - jx, dy = iy - jy, dz = iz - jz;
            if (dx >= -1 && dx <= 1 && dy >= -1 && dy <= 1 && dz >= -1 && dz <= 1) continue;
            if (mode == 1) {
                const int op = c_m2l_lut[(dx + 3) * 49 + (dy + 3) * 7 + (dz + 3)];
                tsrc[w] = (int)cc;
                tdst[w] = (int)b;
                top[w] = op;
                atomicAdd(&lh[op], 1);
                ++w;
            }
            ++c;
        }
    }
    if (mode == 0) count[t] = c;
}

// mode 0: count the M2L pairs of every (target box, parent-neighbour slot);
// mode 1: write them. One thread per (box, slot), so a level's boxes give 27
// times as many threads; the pairs come out ordered by box, then slot.
// Mode 1 also counts the tasks of every operator (hist, kNumM2LOps bins,
// counted per workgroup in LDS first).
__global__ void __launch_bounds__(256) k_m2l_pairs(int mode, int64_t b0, int64_t b1, LevelInfo li,
                                                   const uint64_t *box_key, const int *box_level,
                                                   const int *box_parent, const int *nbr, int *count,
                                                   const int *offs, int *tsrc, int *tdst, int *top, int *hist) {
    __shared__ int lh[kNumM2LOps];
    if (mode == 1) {
        for (int o = threadIdx.x; o < kNumM2LOps; o += blockDim.x) lh[o] = 0;
        __syncthreads();
    }
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t < (b1 - b0) * 27) m2l_pairs_one(mode, t, b0, li, box_key, box_level, box_parent, nbr, count, offs, tsrc,
                                          tdst, top, lh);
    if (mode == 1) {
        __syncthreads();
        for (int o = threadIdx.x; o < kNumM2LOps; o += blockDim.x)
            if (lh[o]) atomicAdd(&hist[o], lh[o]);
    }
}

// Tasks of the M2M/L2L lists of every child level 3..lmax in one pass over
// the boxes b0..b1 of those levels (level by level): child box b <-> its
// parent, operator = the child's octant; hist[8 (level - 3) + octant] counts
// the tasks of every (level, operator), per workgroup in LDS first.
__global__ void __launch_bounds__(256) k_tree_pairs(int64_t b0, int64_t b1, const uint64_t *box_key,
                                                    const int *box_level, const int *box_parent, int nlev,
                                                    int *tsrc, int *tdst, int *top, int *hist) {
    __shared__ int lh[8 * kKeyBits];
    for (int o = threadIdx.x; o < 8 * nlev; o += blockDim.x) lh[o] = 0;
    __syncthreads();
    const int64_t b = b0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (b < b1) {
        const int op = (int)(box_key[b] & 7);
        tsrc[b - b0] = (int)b;
        tdst[b - b0] = box_parent[b];
        top[b - b0] = op;
        atomicAdd(&lh[8 * (box_level[b] - 3) + op], 1);
    }
    __syncthreads();
    for (int o = threadIdx.x; o < 8 * nlev; o += blockDim.x)
        if (lh[o]) atomicAdd(&hist[o], lh[o]);
}

// op_off = exclusive prefix of the per-operator task counts (one workgroup,
// 256 operators at a time); op_off[nops] = the task count.
__global__ void __launch_bounds__(256) k_hist_offsets(const int *hist, int nops, int *op_off) {
    __shared__ int s[256];
    const int tid = threadIdx.x;
    int carry = 0;
    for (int base = 0; base < nops; base += 256) {
        const int o = base + tid;
        const int v = (o < nops) ? hist[o] : 0;
        s[tid] = v;
        __syncthreads();
        for (int d = 1; d < 256; d <<= 1) {
            const int t = (tid >= d) ? s[tid - d] : 0;
            __syncthreads();
            s[tid] += t;
            __syncthreads();
        }
        if (o < nops) op_off[o] = carry + s[tid] - v;
        carry += s[255];
        __syncthreads();
    }
    if (tid == 0) op_off[nops] = carry;
}

// Group by operator keeping the input order within each group: one block
// per operator scans all tasks in order (operator counts are small).
// Tasks of operator blockIdx.x in input order: each thread takes a
// contiguous run of the task list, the runs' match counts are scanned in
// LDS, and every thread writes its matches from its run's offset.
__global__ void __launch_bounds__(1024) k_op_group(const int *top, const int *src, const int *dst, int64_t n,
                                                   const int *op_off, int *osrc, int *odst) {
    __shared__ int cnt[1024];
    const int op = blockIdx.x;
    const int T = blockDim.x, tid = threadIdx.x;
    const int64_t per = (n + T - 1) / T;
    const int64_t i0 = tid * per, i1 = min(n, i0 + per);
    int c = 0;
    for (int64_t i = i0; i < i1; ++i) c += (top[i] == op) ? 1 : 0;
    cnt[tid] = c;
    __syncthreads();
    for (int d = 1; d < T; d <<= 1) {  // inclusive scan of the counts
        const int v = (tid >= d) ? cnt[tid - d] : 0;
        __syncthreads();
        cnt[tid] += v;
        __syncthreads();
    }
    int r = op_off[op] + cnt[tid] - c;
    for (int64_t i = i0; i < i1; ++i)
        if (top[i] == op) {
            osrc[r] = src[i];
            odst[r] = dst[i];
            ++r;
        }
}

__global__ void k_op_keys(const int *top, int64_t n, uint64_t *key, int *idx) {
    int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    key[i] = (uint64_t)top[i];
    idx[i] = (int)i;
}

__global__ void k_invert(const int *order, int64_t n, int *pos) {
    int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r < n) pos[order[r]] = (int)r;
}

// dst_off[k] = first generated M2L task of target box b0 + k (the tasks come
// out ordered by box, then by parent-neighbour slot: 27 slots per box)
__global__ void k_dst_off(const int *offs, int64_t nb, int64_t total, int *dst_off) {
    int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (k < nb) dst_off[k] = offs[27 * k];
    if (k == nb) dst_off[k] = (int)total;
}

__global__ void k_op_gather(const int *order, const int *src, const int *dst, int64_t n, int *osrc, int *odst) {
    int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int i = order[r];
    osrc[r] = src[i];
    odst[r] = dst[i];
}

// Group tasks by operator, keeping the input order within each group: a
// per-operator scan for a few operators, a stable radix sort on the operator
// index for many. The per-operator task counts were formed with the tasks:
// hist_d on the device, hist_h its host copy.
static void group_tasks(TaskList &tl, int nops, const int *tsrc, const int *tdst, const int *top, int64_t n,
                        const int *hist_d, const int *hist_h, Tree::Scratch &scr, hipStream_t st,
                        bool keep_positions = false) {
    BFM_CHECK(nops <= 8192, BFM_EINVAL, "too many translation operators");
    tl.nops = nops;
    tl.ntasks = n;
    tl.op_off_h.assign(nops + 1, 0);
    tl.op_off.ensure(nops + 1);
    for (int c = 0; c < 24; ++c) {
        tl.ntiles[c] = 0;
        tl.tiles_ready[c] = false;
    }
    for (int o = 0; o < nops; ++o) tl.op_off_h[o + 1] = tl.op_off_h[o] + hist_h[o];
    BFM_CHECK(tl.op_off_h[nops] == n, BFM_EDEVICE, "translation task counts disagree");
    k_hist_offsets<<<1, 256, 0, st>>>(hist_d, nops, tl.op_off.get());
    BFM_LAUNCHED();
    tl.src.ensure(n > 0 ? n : 1);
    tl.dst.ensure(n > 0 ? n : 1);
    if (n > 0 && nops <= 16) {
        k_op_group<<<nops, 1024, 0, st>>>(top, tsrc, tdst, n, tl.op_off.get(), tl.src.get(), tl.dst.get());
        BFM_LAUNCHED();
    } else if (n > 0) {
        uint64_t *k0 = scr.ikey.ensure(n), *k1 = scr.ikey2.ensure(n);
        int *i0 = scr.iidx.ensure(n), *i1 = scr.iidx2.ensure(n);
        k_op_keys<<<nblk(n, 256), 256, 0, st>>>(top, n, k0, i0);
        BFM_LAUNCHED();
        int bits = 1;
        while ((1 << bits) < nops) ++bits;
        radix_sort(k0, i0, k1, i1, n, bits, scr, st);
        k_op_gather<<<nblk(n, 256), 256, 0, st>>>(i0, tsrc, tdst, n, tl.src.get(), tl.dst.get());
        BFM_LAUNCHED();
        if (keep_positions) {
            tl.pos_of.ensure(n);
            k_invert<<<nblk(n, 256), 256, 0, st>>>(i0, n, tl.pos_of.get());
            BFM_LAUNCHED();
        }
    }
    BFM_CHECK(!keep_positions || n == 0 || nops > 16, BFM_EINVAL, "task positions kept only for the sorted grouping");
}

// Workgroup-tile prefix of one (channel count, tile width) shape:
// tile_off[o] = sum over o' < o of ceil(cols(o') / width), cols(o) = tasks of
// operator o times nch. One workgroup scans the operators 256 at a time.
__global__ void __launch_bounds__(256) k_tile_off(const int *op_off, int nops, int nch, int width,
                                                  int *tile_off) {
    __shared__ int s[256];
    const int tid = threadIdx.x;
    int carry = 0;
    for (int base = 0; base < nops; base += 256) {
        const int o = base + tid;
        const int v = (o < nops) ? ((op_off[o + 1] - op_off[o]) * nch + width - 1) / width : 0;
        s[tid] = v;
        __syncthreads();
        for (int d = 1; d < 256; d <<= 1) {
            const int t = (tid >= d) ? s[tid - d] : 0;
            __syncthreads();
            s[tid] += t;
            __syncthreads();
        }
        if (o < nops) tile_off[o] = carry + s[tid] - v;
        carry += s[255];
        __syncthreads();
    }
    if (tid == 0) tile_off[nops] = carry;
}

void prepare_tiles(TaskList &tl, int nch, int width, hipStream_t st) {
    BFM_CHECK(nch >= 1 && nch < 8 && (width == 64 || width == 128 || width == 16), BFM_EINVAL,
              "tile shape out of range");
    const int sl = TaskList::slot(nch, width);
    if (tl.tiles_ready[sl]) return;
    // the tile count (the grid size) from the host copy of the operator
    // offsets; the prefix itself is scanned on the device, in stream order, so
    // that the first product of a new tree does not wait for the device
    int run = 0;
    for (int o = 0; o < tl.nops; ++o) {
        const int cols = (tl.op_off_h[o + 1] - tl.op_off_h[o]) * nch;
        run += (cols + width - 1) / width;
    }
    tl.tile_off[sl].ensure(tl.nops + 1);
    k_tile_off<<<1, 256, 0, st>>>(tl.op_off.get(), tl.nops, nch, width, tl.tile_off[sl].get());
    BFM_LAUNCHED();
    tl.ntiles[sl] = run;
    tl.tiles_ready[sl] = true;
}

// ---------------------------------------------------------------------------

__global__ void k_sort_points(const double *xyz, const int *perm, int64_t n, double *px, double *py,
                              double *pz, int *iperm) {
    const int64_t i = xcd_block() * blockDim.x + threadIdx.x;  // neighbouring boxes stay in one L2
    if (i >= n) return;
    const int o = perm[i];
    px[i] = xyz[3 * (int64_t)o];
    py[i] = xyz[3 * (int64_t)o + 1];
    pz[i] = xyz[3 * (int64_t)o + 2];
    iperm[o] = (int)i;
}

__global__ void k_sort_geom(const double *s, const double *nrm, const int *perm, int64_t n,
                            double *ps, double *pnx, double *pny, double *pnz) {
    const int64_t i = xcd_block() * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int o = perm[i];
    ps[i] = s[o];
    pnx[i] = nrm[o];
    pny[i] = nrm[n + o];
    pnz[i] = nrm[2 * n + o];
}


// Host round trips. The build waits for its stream twice: once for the
// level counts (the depth and the box counts size everything after them;
// the bounding cube comes back with them) and once for the sizes of the
// work lists (near-field pair count, largest leaf, item counts, M2L task
// count and the per-operator task counts of every translation list). The
// M2L and M2M/L2L tasks are written before that wait into buffers sized by
// the per-box bounds (at most 216 M2L candidates per box, one M2M task per
// child box). A depth beyond the first sort's ten levels costs a third wait.
namespace {
// layout of the pinned host block the two waits read into
struct HostSizes {
    unsigned long long cnt[kKeyBits + 1];  // boxes per level
    double geo[8];                         // cube (k_bbox_final)
    unsigned long long npairs;             // near-field pairs
    int mo[5];                             // largest leaf, split flag, three item counts
    int m2l_total;
    int hist[kNumM2LOps + 8 * kKeyBits];   // tasks per operator: M2L, then M2M levels 3..lmax
};
}  // namespace

static HostSizes *host_sizes(Tree::Scratch &scr) {
    if (!scr.host) {
        void *p = nullptr;
        BFM_HIP(hipHostMalloc(&p, sizeof(HostSizes), hipHostMallocDefault));
        scr.host = p;
    }
    return static_cast<HostSizes *>(scr.host);
}

void build_tree(Tree &t, const double *xyz, int64_t n, int lmax_req, int leaf_target, int sym_shape,
                hipStream_t st) {
    BFM_CHECK(n >= 1, BFM_EINVAL, "tree of no points");
    BFM_CHECK(sym_shape >= 0 && sym_shape < kSymShapeCount, BFM_EINVAL, "near-field item shape out of range");
    t.valid = false;
    t.n = n;
    const SymShape sh = kSymShapes[sym_shape];
    static_assert(kSymShapes[0].dpiece % 64 == 0 && kSymShapes[1].dpiece % 64 == 0 && kSymShapes[2].dpiece % 64 == 0,
                  "pieces of a chunk's own block start at receiver-group bounds");
    static_assert(kSymShapes[0].chunk <= kSymChunk && kSymShapes[1].chunk <= kSymChunk &&
                      kSymShapes[2].chunk <= kSymChunk && kSymShapes[1].chunk % 64 == 0,
                  "at most four receivers per lane");
    t.sym_shape = sym_shape;
    t.sym_chunk = sh.chunk;
    Tree::Scratch &scr = t.scratch;
    HostSizes *hs = host_sizes(scr);
    // device block: [0, 6 nbb) partial boxes, then the cube (8 doubles)
    const int nbb = 256;
    double *part = scr.bbox.ensure(6 * nbb + 8);
    double *geo = part + 6 * nbb;
    k_bbox_partial<<<nbb, 256, 0, st>>>(xyz, n, part);
    BFM_LAUNCHED();
    k_bbox_final<<<1, 256, 0, st>>>(part, nbb, geo);
    BFM_LAUNCHED();

    // keys + sort
    t.key_a.ensure(n);
    t.key_b.ensure(n);
    t.idx_a.ensure(n);
    t.idx_b.ensure(n);
    k_morton<<<nblk(n, 256), 256, 0, st>>>(xyz, n, geo, t.key_a.get(), t.idx_a.get());
    BFM_LAUNCHED();
    // Sort by the keys' top 30 bits first (levels 1..10: four 8-bit passes
    // instead of six). The boxes of every level <= 10 are then contiguous,
    // which is all an octree of depth <= 10 needs (points inside a level-10
    // box keep their input order); a deeper octree sorts all 45 bits.
    constexpr int kSortedLevels = 10;
    radix_sort_range(t.key_a.get(), t.idx_a.get(), t.key_b.get(), t.idx_b.get(), n,
                     3 * (kKeyBits - kSortedLevels), 3 * kSortedLevels, scr, st);
    int sorted_levels = kSortedLevels;
    DevBuf<int> &tmp = scr.tmp;

    // boxes per level (exact for the sorted levels), read back with the cube
    DevBuf<unsigned long long> &cnt = scr.cnt;
    cnt.ensure(kKeyBits + 1);
    const unsigned long long *ch = hs->cnt;
    auto count_levels = [&]() {
        k_fill_u64<<<1, 64, 0, st>>>(cnt.get(), kKeyBits + 1, 0ull);
        BFM_LAUNCHED();
        k_level_counts<<<std::min(nblk(n, 256), 512u), 256, 0, st>>>(t.key_a.get(), n, kKeyBits, cnt.get());
        BFM_LAUNCHED();
        BFM_HIP(hipMemcpyAsync(hs->cnt, cnt.get(), sizeof(hs->cnt), hipMemcpyDeviceToHost, st));
        BFM_HIP(hipMemcpyAsync(hs->geo, geo, sizeof(hs->geo), hipMemcpyDeviceToHost, st));
        BFM_HIP(hipStreamSynchronize(st));
    };
    // the requested depth, else the deepest sorted level whose mean leaf
    // occupancy is >= leaf_target (at least 2)
    auto pick = [&]() {
        if (lmax_req > 0) return lmax_req;
        int d = 2;
        for (int l = 2; l <= sorted_levels; ++l)
            if ((double)n / (double)ch[l] >= (double)std::max(leaf_target, 1)) d = l;
        return d;
    };
    count_levels();
    BFM_CHECK(hs->geo[5] == 1.0, BFM_EMESH, "non-finite vertex coordinate");
    for (int d = 0; d < 3; ++d) t.origin[d] = hs->geo[d];
    t.side = hs->geo[3];
    int lmax = pick();
    if (lmax > kSortedLevels || (lmax_req <= 0 && lmax == kSortedLevels)) {
        // a deeper octree is asked for, or the occupancy rule may go deeper
        radix_sort(t.key_a.get(), t.idx_a.get(), t.key_b.get(), t.idx_b.get(), n, 3 * kKeyBits, scr, st);
        sorted_levels = kKeyBits;
        count_levels();
        lmax = pick();
    }
    BFM_CHECK(lmax >= 2 && lmax <= kKeyBits, BFM_EINVAL, "octree depth must be in [2, 15]");
    t.lmax = lmax;
    t.lvl_off.assign(lmax + 2, 0);
    for (int l = 0; l <= lmax; ++l) t.lvl_off[l + 1] = t.lvl_off[l] + (int64_t)ch[l];
    t.nbox = t.lvl_off[lmax + 1];
    t.nleaf = (int64_t)ch[lmax];
    LevelInfo li;
    for (int l = 0; l <= kKeyBits + 1; ++l) li.off[l] = (l <= lmax + 1) ? t.lvl_off[l] : t.nbox;
    for (int l = 0; l <= kKeyBits; ++l) li.h[l] = t.side / (double)(1 << l);

    t.box_key.ensure(t.nbox);
    t.box_level.ensure(t.nbox);
    t.box_pt0.ensure(t.nbox + 1);
    t.box_parent.ensure(t.nbox);
    t.box_centre.ensure(3 * t.nbox);
    t.nbr.ensure(27 * t.nbox);
    DevBuf<int> &flag = scr.flag, &pos = scr.pos;
    const int64_t nflag = (int64_t)(lmax + 1) * n;
    BFM_CHECK(nflag < ((int64_t)1 << 31), BFM_EINVAL, "too many points for the octree depth");
    flag.ensure(nflag);
    pos.ensure(nflag);
    t.pt_leaf.ensure(n);
    k_level_flags<<<nblk(nflag, 256), 256, 0, st>>>(t.key_a.get(), n, lmax, flag.get());
    BFM_LAUNCHED();
    exclusive_scan_async(flag.get(), pos.get(), nflag, st, tmp);
    k_level_scatter<<<nblk(nflag, 256), 256, 0, st>>>(t.key_a.get(), n, lmax, flag.get(), pos.get(), t.lvl_off[lmax],
                                                      t.box_key.get(), t.box_level.get(), t.box_pt0.get(),
                                                      t.pt_leaf.get());
    BFM_LAUNCHED();
    k_box_meta<<<nblk(27 * t.nbox, 256), 256, 0, st>>>(t.nbox, lmax, li, t.origin[0], t.origin[1],
                                                       t.origin[2], t.box_key.get(), t.box_level.get(),
                                                       t.box_parent.get(), t.box_centre.get(), t.nbr.get());
    BFM_LAUNCHED();
    // leaves: point ranges, near-field pair count and ranges, and the counts
    // of the work item lists of P2M/L2P, the one-sided and the symmetric near
    // field
    t.leaf_pt.ensure(t.nleaf + 1);
    DevBuf<unsigned long long> &np = scr.np;
    np.ensure(1);
    DevBuf<int> &mo = scr.mo;
    mo.ensure(6);  // largest leaf, some leaf's sources split, three item counts, M2L task count
    k_fill_u64<<<1, 64, 0, st>>>(np.get(), 1, 0ull);
    BFM_LAUNCHED();
    k_fill_int<<<1, 64, 0, st>>>(mo.get(), 6, 0);
    BFM_LAUNCHED();
    k_leaf_near<<<nblk(t.nleaf, 128), 128, 0, st>>>(t.nleaf, t.lvl_off[lmax], t.box_pt0.get(), n,
                                                    t.nbr.get(), t.leaf_pt.get(), np.get(), mo.get());
    BFM_LAUNCHED();
    t.near_rng.ensure(27 * t.nleaf);
    t.near_cnt.ensure(t.nleaf);
    k_leaf_ranges<<<nblk(64 * t.nleaf, 256), 256, 0, st>>>(t.nleaf, t.lvl_off[lmax], t.leaf_pt.get(), t.nbr.get(),
                                                      t.near_rng.get(), t.near_cnt.get());
    BFM_LAUNCHED();
    // counts and offsets: leaf items (icnt, ioff), one-sided near-field
    // pieces (flag, pos; free after the levels, n >= nleaf entries) and
    // symmetric items (lcnt, loff)
    DevBuf<int> &icnt = scr.icnt, &ioff = scr.ioff, &lcnt = scr.lcnt, &loff = scr.loff;
    icnt.ensure(t.nleaf);
    ioff.ensure(t.nleaf);
    lcnt.ensure(t.nleaf);
    loff.ensure(t.nleaf);
    int *pcnt = flag.get(), *poff = pos.get();
    k_item_count<<<nblk(t.nleaf, 256), 256, 0, st>>>(t.nleaf, t.leaf_pt.get(), icnt.get());
    BFM_LAUNCHED();
    k_piece_count<<<nblk(t.nleaf, 256), 256, 0, st>>>(t.nleaf, t.leaf_pt.get(), t.near_rng.get(), t.near_cnt.get(),
                                                     pcnt, mo.get() + 1);
    BFM_LAUNCHED();
    k_sym_items<false><<<nblk(t.nleaf, 256), 256, 0, st>>>(t.nleaf, t.leaf_pt.get(), t.near_rng.get(),
                                                           t.near_cnt.get(), sh, lcnt.get(), nullptr, nullptr);
    BFM_LAUNCHED();
    exclusive_scan_async(icnt.get(), ioff.get(), t.nleaf, st, tmp);
    exclusive_scan_async(pcnt, poff, t.nleaf, st, tmp);
    exclusive_scan_async(lcnt.get(), loff.get(), t.nleaf, st, tmp);
    k_scan_totals3<<<1, 64, 0, st>>>(icnt.get(), ioff.get(), pcnt, poff, lcnt.get(), loff.get(), t.nleaf,
                                     mo.get() + 2);
    BFM_LAUNCHED();

    // M2L tasks over levels 2..lmax, and the per-operator counts
    {
        static int lut_done = 0;  // one bit per device ordinal < 32
        int dev = 0;
        BFM_HIP(hipGetDevice(&dev));
        if (dev >= 32 || !((lut_done >> dev) & 1)) {
            signed short lut[343];
            for (int a = -3; a <= 3; ++a)
                for (int b = -3; b <= 3; ++b)
                    for (int c = -3; c <= 3; ++c)
                        lut[(a + 3) * 49 + (b + 3) * 7 + (c + 3)] = (signed short)m2l_op_index(a, b, c);
            BFM_HIP(hipMemcpyToSymbol(HIP_SYMBOL(c_m2l_lut), lut, sizeof(lut)));
            if (dev < 32) lut_done |= 1 << dev;
        }
    }
    const int nlev = std::max(0, lmax - 2);  // M2M/L2L child levels 3..lmax
    const int nhist = kNumM2LOps + 8 * nlev;
    int *hist = scr.hist.ensure(nhist);
    k_fill_int<<<nblk(nhist, 256), 256, 0, st>>>(hist, nhist, 0);
    BFM_LAUNCHED();
    const int64_t mb0 = t.lvl_off[2], mb1 = t.lvl_off[lmax + 1];
    const int64_t mnb = mb1 - mb0;
    DevBuf<int> &count = scr.count, &offs = scr.offs;
    count.ensure(27 * mnb);
    offs.ensure(27 * mnb);
    k_m2l_pairs<<<nblk(27 * mnb, 256), 256, 0, st>>>(0, mb0, mb1, li, t.box_key.get(), t.box_level.get(),
                                                    t.box_parent.get(), t.nbr.get(), count.get(), nullptr, nullptr,
                                                    nullptr, nullptr, nullptr);
    BFM_LAUNCHED();
    {
        int64_t slot = 0;
        int *sc = scan_scratch(27 * mnb, tmp, &slot);
        int *dtotal = mo.get() + 5;
        k_scan_last<<<1, 64, 0, st>>>(count.get(), 27 * mnb, dtotal);
        BFM_LAUNCHED();
        scan_rec(count.get(), offs.get(), 27 * mnb, st, sc);
        k_scan_total<<<1, 64, 0, st>>>(offs.get(), 27 * mnb, dtotal);
        BFM_LAUNCHED();
    }
    const int64_t m2l_cap = 216 * mnb;  // 27 parent neighbours x 8 children per box
    DevBuf<int> &ts = scr.ts, &td = scr.td, &to = scr.to;
    ts.ensure(m2l_cap + 1);
    td.ensure(m2l_cap + 1);
    to.ensure(m2l_cap + 1);
    k_m2l_pairs<<<nblk(27 * mnb, 256), 256, 0, st>>>(1, mb0, mb1, li, t.box_key.get(), t.box_level.get(),
                                                    t.box_parent.get(), t.nbr.get(), count.get(), offs.get(),
                                                    ts.get(), td.get(), to.get(), hist);
    BFM_LAUNCHED();
    // M2M/L2L tasks of child levels 3..lmax
    const int64_t cb0 = t.lvl_off[std::min(3, lmax + 1)], cb1 = t.lvl_off[lmax + 1];
    DevBuf<int> &cs = scr.cs, &cd = scr.cd, &co = scr.co;
    cs.ensure(cb1 - cb0 + 1);
    cd.ensure(cb1 - cb0 + 1);
    co.ensure(cb1 - cb0 + 1);
    if (cb1 > cb0) {
        k_tree_pairs<<<nblk(cb1 - cb0, 256), 256, 0, st>>>(cb0, cb1, t.box_key.get(), t.box_level.get(),
                                                          t.box_parent.get(), nlev, cs.get(), cd.get(), co.get(),
                                                          hist + kNumM2LOps);
        BFM_LAUNCHED();
    }

    // the second wait: every size the rest needs
    BFM_HIP(hipMemcpyAsync(&hs->npairs, np.get(), sizeof(hs->npairs), hipMemcpyDeviceToHost, st));
    BFM_HIP(hipMemcpyAsync(hs->mo, mo.get(), sizeof(int) * 6, hipMemcpyDeviceToHost, st));
    BFM_HIP(hipMemcpyAsync(hs->hist, hist, sizeof(int) * nhist, hipMemcpyDeviceToHost, st));
    BFM_HIP(hipStreamSynchronize(st));
    t.npairs_near = (int64_t)hs->npairs;
    t.max_leaf = hs->mo[0];
    t.near_split = hs->mo[1] != 0;
    const int64_t ni = hs->mo[2], nn = hs->mo[3], ns = hs->mo[4], total = hs->mo[5];
    BFM_CHECK(total >= 0 && total <= m2l_cap, BFM_EDEVICE, "M2L task count out of range");
    {
        // leaf chunks of at most kLeafChunk points (P2M, L2P)
        t.leaf_items.ensure(ni > 0 ? ni : 1);
        k_item_fill<<<nblk(t.nleaf, 256), 256, 0, st>>>(t.nleaf, t.leaf_pt.get(), ioff.get(), t.leaf_items.get());
        BFM_LAUNCHED();
        t.n_leaf_items = ni;
        // near-field items: leaf chunks x balanced pieces of the source list,
        // in leaf (Morton) order
        t.near_items.ensure(nn > 0 ? nn : 1);
        k_piece_fill<<<nblk(t.nleaf, 256), 256, 0, st>>>(t.nleaf, t.leaf_pt.get(), poff, t.near_rng.get(),
                                                        t.near_cnt.get(), t.near_items.get());
        BFM_LAUNCHED();
        t.n_near_items = nn;
        // symmetric near-field items
        t.sym_items.ensure(ns > 0 ? ns : 1);
        k_sym_items<true><<<nblk(t.nleaf, 256), 256, 0, st>>>(t.nleaf, t.leaf_pt.get(), t.near_rng.get(),
                                                              t.near_cnt.get(), sh, nullptr, loff.get(),
                                                              t.sym_items.get());
        BFM_LAUNCHED();
        t.n_sym_items = ns;
    }
    // M2L lists grouped by operator
    group_tasks(t.m2l, kNumM2LOps, ts.get(), td.get(), to.get(), total, hist, hs->hist, scr, st, true);
    t.m2l.dst_box0 = mb0;
    t.m2l.dst_nbox = mnb;
    t.m2l.dst_off.ensure(mnb + 1);
    k_dst_off<<<nblk(mnb + 1, 256), 256, 0, st>>>(offs.get(), mnb, total, t.m2l.dst_off.get());
    BFM_LAUNCHED();
    // M2M / L2L lists: child levels 3..lmax (index l)
    // task lists are reused between builds (their buffers only grow)
    for (size_t l = lmax + 1; l < t.m2m.size(); ++l) {
        delete t.m2m[l];
        t.m2m[l] = nullptr;
    }
    t.m2m.resize(lmax + 1, nullptr);
    for (int l = 3; l <= lmax; ++l) {
        const int64_t o = t.lvl_off[l] - cb0, nb = t.lvl_off[l + 1] - t.lvl_off[l];
        const int hk = kNumM2LOps + 8 * (l - 3);
        if (!t.m2m[l]) t.m2m[l] = new TaskList();
        group_tasks(*t.m2m[l], 8, cs.get() + o, cd.get() + o, co.get() + o, nb, hist + hk, hs->hist + hk, scr, st);
    }
    // sorted positions
    t.iperm.ensure(n);
    t.px.ensure(n);
    t.py.ensure(n);
    t.pz.ensure(n);
    k_sort_points<<<nblk(n, 256), 256, 0, st>>>(xyz, t.idx_a.get(), n, t.px.get(), t.py.get(),
                                                t.pz.get(), t.iperm.get());
    BFM_LAUNCHED();
    t.valid = true;  // (the work above stays in flight: later launches are stream-ordered)
}

void sort_geometry(Tree &t, const double *s, const double *nrm, hipStream_t st) {
    const int64_t n = t.n;
    t.ps.ensure(n);
    t.pnx.ensure(n);
    t.pny.ensure(n);
    t.pnz.ensure(n);
    k_sort_geom<<<nblk(n, 256), 256, 0, st>>>(s, nrm, t.idx_a.get(), n, t.ps.get(), t.pnx.get(),
                                              t.pny.get(), t.pnz.get());
    BFM_LAUNCHED();
}

}  // namespace bfm
