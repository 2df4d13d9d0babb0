// polygon.hip - isochrone polygons on the device: the border of the region in range traced
// along the faces of a planar embedding (Section 7).
//
// The embedding is a rotation system built once per graph on the host from the vertex
// coordinates: every undirected neighbour pair {u, v} of the input gives two darts (u, v) and
// (v, u); dart ids are the darts in (u, v) order over original ids, and around every vertex
// the darts are ordered counterclockwise by the angle of the straight segment to the
// neighbour (equal angles by neighbour id).  Tracing the face on the left of a dart (a, b)
// continues with (b, c), c the neighbour of b next clockwise from a: fnext[] holds that step.
//
// A query runs the vertex-output sweep of k <= 64 queries (lane masks of the vertices in
// range by position), then per lane:
//   1. the boundary darts (u in range, v not), as (lane, dart) keys, sorted;
//   2. from each boundary dart, the walk along its face up to the first dart that enters the
//      region; that dart's twin is the next boundary dart of the border (pointer `nxt`);
//   3. the cycles of nxt: every dart's cycle minimum and its distance to it, by pointer
//      doubling (one workgroup per lane);
//   4. cycles listed from their smallest dart, in the order of those, by one exclusive scan.
// All per-lane work is on the device; the host copies the result out.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>

#include "device.h"

namespace isodev {

#define PCHK(x)                                                                     \
    do {                                                                            \
        hipError_t _e = (x);                                                        \
        if (_e != hipSuccess) {                                                     \
            set_error(std::string(#x) + ": " + hipGetErrorString(_e));              \
            return -3;                                                              \
        }                                                                           \
    } while (0)

constexpr uint32_t POLY_CYC_THREADS = 1024;

__device__ __forceinline__ void pswap(uint32_t *&a, uint32_t *&b) {
    uint32_t *t = a;
    a = b;
    b = t;
}

// ------------------------------------------------------------------------------ kernels

// Step 1: boundary darts.  One thread per original vertex u (waves stay whole through the
// loop); a wavefront sums its threads' counts and claims its output range with one atomic.
__global__ void k_poly_darts(const uint32_t *__restrict__ off, const uint32_t *__restrict__ hpos,
                             const uint32_t *__restrict__ pos, const uint64_t *__restrict__ vmask, uint32_t n,
                             uint64_t lanes_mask, uint64_t *__restrict__ keys, uint32_t *__restrict__ count,
                             uint32_t cap) {
    const uint64_t total = (uint64_t(n) + 63u) & ~uint64_t(63);
    const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
    const uint32_t lane = __lane_id();
    for (uint64_t t = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < total; t += stride) {
        const uint32_t u = uint32_t(t);
        uint64_t mu = 0;
        uint32_t e0 = 0, e1 = 0;
        if (u < n) {
            mu = vmask[pos[u]] & lanes_mask;
            if (mu) {
                e0 = off[u];
                e1 = off[u + 1];
            }
        }
        uint32_t c = 0;
        for (uint32_t k = e0; k < e1; ++k) c += __popcll(mu & ~vmask[hpos[k]]);
        // inclusive scan of the counts over the wavefront
        uint32_t incl = c;
        for (uint32_t d = 1; d < 64; d <<= 1) {
            const uint32_t y = __shfl_up(incl, d, 64);
            if (lane >= d) incl += y;
        }
        const uint32_t wsum = __shfl(incl, 63, 64);
        uint32_t base = 0;
        if (lane == 63 && wsum) base = atomicAdd(count, wsum);
        base = __shfl(base, 63, 64);
        uint32_t o = base + incl - c;
        for (uint32_t k = e0; k < e1 && c; ++k)
            for (uint64_t b = mu & ~vmask[hpos[k]]; b; b &= b - 1u, ++o)
                if (o < cap) keys[o] = (uint64_t(__builtin_ctzll(b)) << 32) | k;
    }
}

// First index of lane j's keys (j = 0..lanes): keys are sorted by (lane, dart).
__global__ void k_poly_lane_off(const uint64_t *__restrict__ keys, uint32_t cnt, uint32_t lanes,
                                uint32_t *__restrict__ loff) {
    const uint32_t j = threadIdx.x;
    if (j > lanes) return;
    const uint64_t want = uint64_t(j) << 32;
    uint32_t lo = 0, hi = cnt;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (keys[mid] < want) lo = mid + 1; else hi = mid;
    }
    loff[j] = lo;
}

// Step 2: the successor of every boundary dart.  From (u, v) (u in, v out) the face on its
// left is walked until a dart (a, b) with a out of range and b in range; its twin (b, a) is a
// boundary dart, found by binary search in the lane's sorted keys.  The walk ends within the
// face's length (the face returns to u, which is in range); `limit` only guards the loop.
__global__ void k_poly_next(const uint64_t *__restrict__ keys, uint32_t cnt, const uint32_t *__restrict__ loff,
                            const uint32_t *__restrict__ fnext, const uint32_t *__restrict__ twin,
                            const uint32_t *__restrict__ hpos, const uint64_t *__restrict__ vmask, uint64_t limit,
                            uint32_t *__restrict__ nxt, uint32_t *__restrict__ err) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cnt) return;
    const uint64_t key = keys[i];
    const uint32_t j = uint32_t(key >> 32);
    uint32_t kk = uint32_t(key);
    bool in_a = false;   // the head of the starting dart is out of range
    for (uint64_t step = 0;; ++step) {
        kk = fnext[kk];
        const bool in_b = (vmask[hpos[kk]] >> j) & 1ull;
        if (!in_a && in_b) break;
        in_a = in_b;
        if (step >= limit) {
            atomicOr(err, 1u);
            nxt[i] = i;
            return;
        }
    }
    const uint64_t want = (uint64_t(j) << 32) | twin[kk];
    uint32_t lo = loff[j], hi = loff[j + 1];
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (keys[mid] < want) lo = mid + 1; else hi = mid;
    }
    if (lo < loff[j + 1] && keys[lo] == want) {
        nxt[i] = lo;
    } else {
        atomicOr(err, 2u);
        nxt[i] = i;
    }
}

// Step 3: one workgroup per lane over its darts [loff[j], loff[j+1]).  Pointer doubling over
// nxt gives every dart the smallest index on its cycle (mn), then, with the cycle broken at
// that minimum, the number of steps from the dart to it (rk; Wyllie's list ranking).  A
// cycle's minimum also gets its scan word: 1 << 32 | cycle length.  a0/a1, b0/b1 are
// double buffers of the doubling rounds (cnt words each).
__global__ void __launch_bounds__(POLY_CYC_THREADS)
k_poly_cycles(const uint32_t *__restrict__ loff, const uint32_t *__restrict__ nxt, uint32_t *mn, uint32_t *rk,
              uint32_t *a0, uint32_t *a1, uint32_t *b0, uint32_t *b1, uint64_t *__restrict__ scan,
              const uint32_t *__restrict__ err) {
    const uint32_t j = blockIdx.x, tid = threadIdx.x, T = blockDim.x;
    const uint32_t lo = loff[j], hi = loff[j + 1], L = hi - lo;
    if (L == 0 || *err) return;   // nxt is a permutation of the lane's darts only without an error
    const uint32_t rounds = L <= 1 ? 0u : 32u - __builtin_clz(L - 1u);   // 2^rounds >= L
    // minimum over the cycle: a = running minimum, b = jump pointer
    uint32_t *ma = a0, *mb = a1, *pa = b0, *pb = b1;
    for (uint32_t i = lo + tid; i < hi; i += T) {
        ma[i] = i;
        pa[i] = nxt[i];
    }
    __syncthreads();
    for (uint32_t r = 0; r < rounds; ++r) {
        for (uint32_t i = lo + tid; i < hi; i += T) {
            const uint32_t p = pa[i];
            mb[i] = min(ma[i], ma[p]);
            pb[i] = pa[p];
        }
        __syncthreads();
        pswap(ma, mb);
        pswap(pa, pb);
    }
    for (uint32_t i = lo + tid; i < hi; i += T) mn[i] = ma[i];
    __syncthreads();
    // steps to the cycle's minimum: the minimum absorbs (points to itself, weight 0)
    uint32_t *va = a0, *vb = a1;
    pa = b0;
    pb = b1;
    for (uint32_t i = lo + tid; i < hi; i += T) {
        const bool head = mn[i] == i;
        va[i] = head ? 0u : 1u;
        pa[i] = head ? i : nxt[i];
    }
    __syncthreads();
    for (uint32_t r = 0; r < rounds; ++r) {
        for (uint32_t i = lo + tid; i < hi; i += T) {
            const uint32_t p = pa[i];
            vb[i] = va[i] + va[p];
            pb[i] = pa[p];
        }
        __syncthreads();
        pswap(va, vb);
        pswap(pa, pb);
    }
    for (uint32_t i = lo + tid; i < hi; i += T) rk[i] = va[i];
    __syncthreads();
    // the dart after a minimum is len - 1 steps from it
    for (uint32_t i = lo + tid; i < hi; i += T)
        scan[i] = mn[i] == i ? ((uint64_t(1) << 32) | (uint64_t(rk[nxt[i]]) + 1u)) : 0ull;
}

// Step 4: every dart to its place.  scx is the exclusive scan of `scan`: at a cycle's minimum,
// the cycles before it (high word) and the darts before it (low word).  A dart rk steps before
// the minimum sits len - rk places after it.  Darts are written as (tail, head) original ids,
// and each cycle's start into cyc.
__global__ void k_poly_out(const uint64_t *__restrict__ keys, uint32_t cnt, const uint32_t *__restrict__ mn,
                           const uint32_t *__restrict__ rk, const uint64_t *__restrict__ scan,
                           const uint64_t *__restrict__ scx, const uint32_t *__restrict__ off,
                           const uint32_t *__restrict__ hid, uint32_t n, uint2 *__restrict__ out,
                           uint32_t *__restrict__ cyc, const uint32_t *__restrict__ err) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cnt || *err) return;
    const uint32_t k = uint32_t(keys[i]), m = mn[i];
    const uint32_t len = uint32_t(scan[m]), base = uint32_t(scx[m]);
    const uint32_t p = base + (i == m ? 0u : len - rk[i]);
    uint32_t lo = 0, hi = n;   // tail: the last u with off[u] <= k
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (off[mid] <= k) lo = mid; else hi = mid - 1;
    }
    out[p] = make_uint2(lo, hid[k]);
    if (i == m) cyc[uint32_t(scx[m] >> 32)] = base;
}

// First cycle of every lane (j = 0..lanes; lanes: the total).
__global__ void k_poly_lane_cyc(const uint32_t *__restrict__ loff, const uint64_t *__restrict__ scan,
                                const uint64_t *__restrict__ scx, uint32_t cnt, uint32_t lanes,
                                uint32_t *__restrict__ lcyc) {
    const uint32_t j = threadIdx.x;
    if (j > lanes) return;
    const uint32_t total = cnt ? uint32_t((scx[cnt - 1] + scan[cnt - 1]) >> 32) : 0u;
    const uint32_t i = loff[j];
    lcyc[j] = i < cnt ? uint32_t(scx[i] >> 32) : total;
}

// ------------------------------------------------------------------------------ host

void Rotation::release() {
    void *ptrs[] = {d_off, d_hpos, d_hid, d_twin, d_fnext};
    for (void *p : ptrs) if (p) hipFree(p);
    *this = Rotation();
}

void PolyBufs::release() {
    void *ptrs[] = {d_keys, d_keys2, d_sort_tmp, d_nxt, d_mn, d_rk, d_w, d_scan, d_scx, d_scan_tmp, d_out, d_cyc,
                    d_small};
    for (void *p : ptrs) if (p) hipFree(p);
    *this = PolyBufs();
}

static int grow(void **p, size_t &have, size_t want) {
    if (want <= have && *p) return 0;
    if (*p) hipFree(*p);
    *p = nullptr;
    have = 0;
    if (hipMalloc(p, std::max<size_t>(want, 256)) != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        set_error("device allocation for the polygon buffers failed");
        return -2;
    }
    have = std::max<size_t>(want, 256);
    return 0;
}

template <class F>
static void parallel_for(uint32_t n, int threads, F f) {
    const int T = std::max(1, std::min<int>(threads, int((n + 4095) / 4096)));
    if (T == 1) {
        f(0u, n);
        return;
    }
    std::vector<std::thread> th;
    for (int t = 0; t < T; ++t) {
        const uint32_t a = uint32_t(uint64_t(n) * t / T), b = uint32_t(uint64_t(n) * (t + 1) / T);
        th.emplace_back([=] { f(a, b); });
    }
    for (auto &x : th) x.join();
}

int DevGraph::upload_rotation(const iso::Prep &P, const double *xy, int threads) {
    if (rot.ready) return 0;
    const uint32_t N = P.n;
    for (size_t i = 0; i < 2 * size_t(N); ++i)
        if (!std::isfinite(xy[i])) {
            set_error("vertex coordinates must be finite");
            return -1;
        }
    // undirected neighbour pairs: every downward entry that stands for an original arc, in
    // either direction (both endpoints are then neighbours in the input)
    std::vector<uint64_t> off(size_t(N) + 1, 0);
    for (uint32_t v = 0; v < N; ++v)
        for (uint32_t e = P.down_off[v]; e < P.down_off[v + 1]; ++e) {
            const uint32_t w0 = P.down_arc[2 * uint64_t(e)];
            if (!(w0 & (iso::FLAG_FWD | iso::FLAG_REV))) continue;
            const uint32_t a = P.perm[w0 & iso::TAIL_MASK], b = P.perm[v];
            if (a == b) continue;
            off[a + 1]++;
            off[b + 1]++;
        }
    for (uint32_t v = 0; v < N; ++v) off[v + 1] += off[v];
    std::vector<uint32_t> nb(std::max<uint64_t>(1, off[N]));
    {
        std::vector<uint64_t> fill(off.begin(), off.end() - 1);
        for (uint32_t v = 0; v < N; ++v)
            for (uint32_t e = P.down_off[v]; e < P.down_off[v + 1]; ++e) {
                const uint32_t w0 = P.down_arc[2 * uint64_t(e)];
                if (!(w0 & (iso::FLAG_FWD | iso::FLAG_REV))) continue;
                const uint32_t a = P.perm[w0 & iso::TAIL_MASK], b = P.perm[v];
                if (a == b) continue;
                nb[fill[a]++] = b;
                nb[fill[b]++] = a;
            }
    }
    // per vertex: neighbours by id without repeats (the dart ids), packed to the front
    std::vector<uint32_t> deg(N, 0);
    parallel_for(N, threads, [&](uint32_t a, uint32_t b) {
        for (uint32_t u = a; u < b; ++u) {
            uint32_t *p = nb.data() + off[u], *q = nb.data() + off[u + 1];
            std::sort(p, q);
            deg[u] = uint32_t(std::unique(p, q) - p);
        }
    });
    std::vector<uint64_t> doff(size_t(N) + 1, 0);
    for (uint32_t u = 0; u < N; ++u) doff[u + 1] = doff[u] + deg[u];
    const uint64_t D = doff[N];
    if (D >= uint64_t(iso::INF)) {
        set_error("more than 2^32 - 2 darts: too many edges for the polygon output");
        return -1;
    }
    std::vector<uint32_t> hid(std::max<uint64_t>(1, D));
    for (uint32_t u = 0; u < N; ++u) std::memcpy(hid.data() + doff[u], nb.data() + off[u], deg[u] * 4ull);
    nb.clear();
    nb.shrink_to_fit();
    std::vector<uint32_t> off32(size_t(N) + 1), hpos(std::max<uint64_t>(1, D)), twin(hid.size()),
        cwprev(hid.size()), fnext(hid.size());
    for (uint32_t u = 0; u <= N; ++u) off32[u] = uint32_t(doff[u]);
    parallel_for(N, threads, [&](uint32_t a, uint32_t b) {
        std::vector<std::pair<double, uint32_t>> ang;
        std::vector<uint32_t> ord;
        for (uint32_t u = a; u < b; ++u) {
            const uint32_t k0 = off32[u], d = off32[u + 1] - k0;
            ang.resize(d);
            ord.resize(d);
            for (uint32_t i = 0; i < d; ++i) {
                const uint32_t v = hid[k0 + i];
                hpos[k0 + i] = P.pos[v];
                ang[i] = {std::atan2(xy[2 * size_t(v) + 1] - xy[2 * size_t(u) + 1],
                                     xy[2 * size_t(v)] - xy[2 * size_t(u)]),
                          v};
                // twin: u in v's id-sorted list
                const uint32_t *p = hid.data() + off32[v], *q = hid.data() + off32[v + 1];
                twin[k0 + i] = uint32_t(std::lower_bound(p, q, u) - hid.data());
                ord[i] = i;
            }
            // counterclockwise order (angle, then neighbour id); a dart's clockwise neighbour
            // is the one before it in that order, cyclically
            std::sort(ord.begin(), ord.end(), [&](uint32_t x, uint32_t y) { return ang[x] < ang[y]; });
            for (uint32_t r = 0; r < d; ++r) cwprev[k0 + ord[r]] = k0 + ord[r == 0 ? d - 1 : r - 1];
        }
    });
    parallel_for(uint32_t(D), threads, [&](uint32_t a, uint32_t b) {
        for (uint32_t k = a; k < b; ++k) fnext[k] = cwprev[twin[k]];
    });
    PCHK(hipSetDevice(device));
    Rotation R;
    R.darts = D;
    auto up = [&](uint32_t **dst, const std::vector<uint32_t> &src) -> int {
        PCHK(hipMalloc((void **)dst, src.size() * 4));
        PCHK(hipMemcpy(*dst, src.data(), src.size() * 4, hipMemcpyHostToDevice));
        return 0;
    };
    int r;
    if ((r = up(&R.d_off, off32)) || (r = up(&R.d_hpos, hpos)) || (r = up(&R.d_hid, hid)) ||
        (r = up(&R.d_twin, twin)) || (r = up(&R.d_fnext, fnext))) {
        R.release();
        (void)hipGetLastError();
        return r;
    }
    R.bytes = (off32.size() + 4 * hid.size()) * 4;
    R.ready = true;
    rot = R;
    bytes += R.bytes;
    return 0;
}

int DevGraph::polygons(SweepCtx &C, uint32_t lanes, PolyResult &out) {
    if (!rot.ready || !C.bufs.d_vmask) {
        set_error("polygon: no rotation system or vertex masks");
        return -1;
    }
    PCHK(hipSetDevice(device));
    hipStream_t s = C.stream;
    PolyBufs &B = poly;
    int r;
    // small words: [0] dart count, [1] error flags, [2 .. 2 + 65) lane starts, then 65 lane cycle starts
    if ((r = grow((void **)&B.d_small, B.sz_small, (2 + 2 * (MAX_LANES + 1)) * 4))) return r;
    uint32_t *d_cnt = B.d_small, *d_err = B.d_small + 1, *d_loff = B.d_small + 2,
             *d_lcyc = B.d_small + 2 + MAX_LANES + 1;
    const uint64_t lanes_mask = lanes >= 64 ? ~0ull : ((1ull << lanes) - 1ull);
    uint32_t cnt = 0;
    for (int pass = 0; pass < 2; ++pass) {
        if ((r = grow((void **)&B.d_keys, B.sz_keys, B.cap * 8))) return r;
        PCHK(hipMemsetAsync(B.d_small, 0, 8, s));
        k_poly_darts<<<dim3(std::min<uint32_t>(8192, (n + 255) / 256)), dim3(256), 0, s>>>(
            rot.d_off, rot.d_hpos, d_pos, C.bufs.d_vmask, n, lanes_mask, B.d_keys, d_cnt, uint32_t(B.cap));
        PCHK(hipGetLastError());
        PCHK(hipMemcpyAsync(&cnt, d_cnt, 4, hipMemcpyDeviceToHost, s));
        PCHK(hipStreamSynchronize(s));
        if (cnt <= B.cap) break;
        B.cap = size_t(cnt) + cnt / 4;   // grow and enumerate again (the masks are unchanged)
    }
    if (cnt > B.cap) {
        set_error("polygon: boundary darts changed between two enumerations");
        return -3;
    }
    if (cnt >= (1u << 31)) {
        set_error("polygon: more than 2^31 boundary darts in one sweep");
        return -2;
    }
    out.loff.assign(lanes + 1, 0);
    out.lcyc.assign(lanes + 1, 0);
    out.darts.clear();
    out.cyc.clear();
    if (cnt == 0) return 0;
    const size_t c = cnt;
    if ((r = grow((void **)&B.d_keys2, B.sz_keys2, c * 8)) || (r = grow((void **)&B.d_nxt, B.sz_nxt, c * 4)) ||
        (r = grow((void **)&B.d_mn, B.sz_mn, c * 4)) || (r = grow((void **)&B.d_rk, B.sz_rk, c * 4)) ||
        (r = grow((void **)&B.d_w, B.sz_w, c * 16)) || (r = grow((void **)&B.d_scan, B.sz_scan, c * 8)) ||
        (r = grow((void **)&B.d_scx, B.sz_scx, c * 8)) || (r = grow((void **)&B.d_out, B.sz_out, c * 8)) ||
        (r = grow((void **)&B.d_cyc, B.sz_cyc, c * 4)))
        return r;
    size_t sort_bytes = 0, scan_bytes = 0;
    PCHK(hipcub::DeviceRadixSort::SortKeys(nullptr, sort_bytes, B.d_keys, B.d_keys2, int(c), 0, 38, s));
    PCHK(hipcub::DeviceScan::ExclusiveSum(nullptr, scan_bytes, B.d_scan, B.d_scx, int(c), s));
    if ((r = grow(&B.d_sort_tmp, B.sz_sort_tmp, sort_bytes)) || (r = grow(&B.d_scan_tmp, B.sz_scan_tmp, scan_bytes)))
        return r;
    PCHK(hipcub::DeviceRadixSort::SortKeys(B.d_sort_tmp, sort_bytes, B.d_keys, B.d_keys2, int(c), 0, 38, s));
    k_poly_lane_off<<<dim3(1), dim3(128), 0, s>>>(B.d_keys2, cnt, lanes, d_loff);
    k_poly_next<<<dim3(uint32_t((c + 255) / 256)), dim3(256), 0, s>>>(
        B.d_keys2, cnt, d_loff, rot.d_fnext, rot.d_twin, rot.d_hpos, C.bufs.d_vmask, rot.darts + 2, B.d_nxt, d_err);
    uint32_t *w = B.d_w;
    k_poly_cycles<<<dim3(lanes), dim3(POLY_CYC_THREADS), 0, s>>>(d_loff, B.d_nxt, B.d_mn, B.d_rk, w, w + c,
                                                                 w + 2 * c, w + 3 * c, B.d_scan, d_err);
    PCHK(hipcub::DeviceScan::ExclusiveSum(B.d_scan_tmp, scan_bytes, B.d_scan, B.d_scx, int(c), s));
    k_poly_out<<<dim3(uint32_t((c + 255) / 256)), dim3(256), 0, s>>>(B.d_keys2, cnt, B.d_mn, B.d_rk, B.d_scan,
                                                                   B.d_scx, rot.d_off, rot.d_hid, n, B.d_out, B.d_cyc,
                                                                   d_err);
    k_poly_lane_cyc<<<dim3(1), dim3(128), 0, s>>>(d_loff, B.d_scan, B.d_scx, cnt, lanes, d_lcyc);
    PCHK(hipGetLastError());
    uint32_t small[2 + 2 * (MAX_LANES + 1)];
    PCHK(hipMemcpyAsync(small, B.d_small, sizeof(small), hipMemcpyDeviceToHost, s));
    PCHK(hipStreamSynchronize(s));
    if (small[1]) {
        set_error("polygon: a face walk did not reach a boundary dart");   // not expected: see k_poly_next
        return -3;
    }
    for (uint32_t j = 0; j <= lanes; ++j) {
        out.loff[j] = small[2 + j];
        out.lcyc[j] = small[2 + MAX_LANES + 1 + j];
    }
    const uint32_t ncyc = out.lcyc[lanes];
    out.darts.resize(2 * c);
    out.cyc.resize(ncyc);
    PCHK(hipMemcpyAsync(out.darts.data(), B.d_out, c * 8, hipMemcpyDeviceToHost, s));
    if (ncyc) PCHK(hipMemcpyAsync(out.cyc.data(), B.d_cyc, size_t(ncyc) * 4, hipMemcpyDeviceToHost, s));
    PCHK(hipStreamSynchronize(s));
    return 0;
}

}  // namespace isodev
