// The MPdist-profile kernel: eqs. 9-13 of section 4.1 for every (query, window).
//
// For query s (a segment S_s of T, eq. 4, or an external query Q) the kernel
// evaluates the distance matrix ED_matr (eq. 9) between the query's w = m-l+1
// length-l subsequences (rows) and the series' length-l subsequences
// (columns), its column minima allP_BA (eq. 10), its row minima over a sliding
// window of w columns allP_AB (eq. 11), and for every length-m window j the
// k-th smallest element of the concatenation P_ABBA (eqs. 12-13).
//
// Every later step is an order statistic, monotone in the Pearson correlation
// rho of the two subsequences, because d = sqrt(2 l (1 - rho)).  The kernel
// therefore works on y = (1 - rho) / 2, clamped to [0, 1] (d^2 = 4 l y), and
// forms one distance per window, from the selected y.  Clamped y values are
// non-negative floats, ordered like their bit patterns, so minima, comparisons
// and sorting run on the bits as unsigned integers.
//
// Work unit: a tile of (query, JT consecutive windows), JT = 31 * (number of
// selection threads).  The tile is computed in sub-tiles of SBW windows; a
// sub-tile needs the w x (SBW + w - 1) block of the matrix:
//   1. FP64 anchors: the centred covariance at the first cell of each diagonal
//      of the block, by a direct dot product (register-blocked along the row).
//   2. Rows in chunks of 8: each thread owns V adjacent diagonals and advances
//      them one row at a time with the FP32 centred-covariance recurrence
//          cov(r+1, c+1) = cov(r, c) + df[r]*dg[c] + df[c]*dg[r];
//      the statistics of its V columns sit in a register window that slides by
//      one column per row.  The chunk's y values go to LDS.
//   3. Column minima of y (eq. 10) accumulate in LDS for the sub-tile and go
//      to a per-workgroup copy for the tile.
//   4. Sliding row minima of width w (eq. 11): wave r takes row r of the chunk,
//      lane a the 31 windows of block a: suffix minima of the block and running
//      minima of the window tails in registers, whole blocks in between from
//      block minima the wave shares in LDS.  They go to a per-workgroup scratch
//      slot, laid out so that a wave's stores and loads are contiguous.
//   5. Selection (eqs. 12-13): thread a takes the 31 windows of block a, in
//      order.  A run starts with a per-thread MSD radix select on the bits of y
//      that brackets the ranks k-8 .. k+8; each window then makes one pass that
//      counts the values below the bracket and collects the ones inside it
//      (adjacent windows share all but a few of their 2w values, so the k-th
//      value rarely leaves the bracket), sorts the few collected values and
//      takes the next bracket from them.  A window whose bracket misses gets a
//      second pass with a bracket re-aimed from the first (taken by the
//      missing lanes of a wave together when there are a few of them); what
//      still misses is solved by the 64 lanes of the wave together, one window
//      at a time (by counting ranks for short windows, a radix select for
//      longer ones), so a rare miss costs the wave a short step instead of
//      stalling every lane.  The result is exact either way.
//
// Arithmetic of a cell depends only on the query's data, the column and the
// window offset inside the tile, never on the query's position, so identical
// segments get bit-identical profiles.
#include "pst_internal.h"

#include <algorithm>
#include <atomic>

#include <math.h>

// A build with -DPST_PROBE (build.py --probe, libpst_probe.so) measures, per
// profile launch, the wave time of each phase and how often the selection's
// paths run (pst_probe_read); the counters cost time and are for analysis only.
#ifdef PST_PROBE
// counter i is spread over 64 addresses (by lane, or by wave for the times)
__device__ unsigned long long g_probe[32 * 64];
#define PROBE(i, c) atomicAdd(&g_probe[(i) * 64 + (threadIdx.x & 63)], (unsigned long long)(c))
// wave time between two marks, by lane 0 of the wave
#define PROBE_MARK(v) const long long v = clock64()
#define PROBE_SPAN(i, v)                                                                              \
    do {                                                                                              \
        if ((threadIdx.x & 63) == 0)                                                                  \
            atomicAdd(&g_probe[(i) * 64 + ((blockIdx.x * 8 + (threadIdx.x >> 6)) & 63)],               \
                      (unsigned long long)(clock64() - (v)));                                         \
    } while (0)
#else
#define PROBE(i, c) ((void)0)
#define PROBE_MARK(v) ((void)0)
#define PROBE_SPAN(i, v) ((void)0)
#endif

namespace pst {
namespace {

constexpr int G = 31;      // windows per block (odd: conflict-free LDS strides)
constexpr int kStageIters = 5;   // column-statistics entries per thread per sub-tile, at most
constexpr int CAP = 28;    // sorted candidate list capacity
constexpr int NB = 16;     // radix buckets per level
constexpr int BAND = 8;    // bracket half-width in ranks
// A wave runs the second bracket pass only when at least this many of its
// lanes missed: the pass costs the whole wave a pass, a cooperative select
// costs it a fraction of one (thresholds 1, 2, 3, 4 and 6 measured on w = 33
// .. 513: 3 and 4 fastest, 1 up to 9 % slower).
constexpr int RETRY_MIN = 3;
constexpr int BL = 32;     // values per load batch of a window pass
constexpr int BMW = 128;   // block minima per row (two blocks per lane at most)
constexpr int RPAD = 32;   // LDS floats after the row buffer (row-minimum reads past a row end)

struct Geo {
    int NT;     // threads per workgroup (512, or 256 with two workgroups per CU)
    int JT;     // windows per tile
    int nA;     // selection threads = blocks per tile = JT / G
    int SBW;    // windows per sub-tile (multiple of G)
    int V;      // diagonals per thread
    int RCH;    // rows per chunk (8, or 4 where LDS is short)
};

struct ProfileArgs {
    ProfileBatch B;
    Geo g;
};

__device__ __forceinline__ uint32_t key_of(float y) { return __float_as_uint(y); }
// Minimum of two non-negative floats (or +inf) through their bit patterns.
__device__ __forceinline__ float umin(float a, float b) {
    return __uint_as_float(min(__float_as_uint(a), __float_as_uint(b)));
}

// Sorts a[0..N) ascending with Batcher's odd-even merge network (truncated to
// N inputs: the missing inputs would be the largest keys and never move).
template <int N>
__device__ __forceinline__ void sort_net(uint32_t (&a)[N]) {
#pragma unroll
    for (int p = 1; p < N; p += p) {
#pragma unroll
        for (int k = p; k > 0; k /= 2) {
#pragma unroll
            for (int j = k % p; j + k < N; j += 2 * k) {
#pragma unroll
                for (int i = 0; i < k; ++i) {
                    if (i + j + k < N && (i + j) / (2 * p) == (i + j + k) / (2 * p)) {
                        const uint32_t x = a[i + j], y = a[i + j + k];
                        a[i + j] = min(x, y);
                        a[i + j + k] = max(x, y);
                    }
                }
            }
        }
    }
}

// One thread's pass over the 2w values of a window: first A(i), i < w, the
// row minima in the scratch buffer R (row i at byte offset voff + i * rstr);
// then B(c) = bv[c], c < w, from LDS.  f(key, valid) sees every value once.
// Values go in batches of BL, loads a batch ahead of use; the last batch of
// each half stops at the group of GQ values that holds the half's end (w is
// the same for the whole wave, so those checks are scalar branches), and its
// padding values come with valid = false.  w = m/2 + 1 lies just past a
// multiple of BL for the usual lengths, so whole padded batches would
// almost double the work of short windows.
constexpr int GQ = 8;
template <typename F>
__device__ __forceinline__ void window_pass(__amdgpu_buffer_rsrc_t R, uint32_t voff, uint32_t rstr, const float *bv,
                                            int w, F &&f) {
    const int wm1 = w - 1;
    auto load_full = [&](uint32_t (&y)[BL], int i0) {  // rows i0 .. i0+BL-1, all inside
#pragma unroll
        for (int e = 0; e < BL; ++e)
            y[e] = __builtin_amdgcn_raw_buffer_load_b32(R, (int)voff, (int)((uint32_t)(i0 + e) * rstr), 0);
    };
    auto load = [&](uint32_t (&y)[BL], int i0) {  // a batch that may hold the end
        const int lim = w - i0;
#pragma unroll
        for (int q = 0; q < BL / GQ; ++q) {
            if (q * GQ < lim) {
#pragma unroll
                for (int e = q * GQ; e < q * GQ + GQ; ++e) {
                    const int i = min(i0 + e, wm1);
                    y[e] = __builtin_amdgcn_raw_buffer_load_b32(R, (int)voff, (int)((uint32_t)i * rstr), 0);
                }
            }
        }
    };
    auto use = [&](const uint32_t (&y)[BL], int lim) {
#pragma unroll
        for (int q = 0; q < BL / GQ; ++q) {
            if (q * GQ < lim) {
#pragma unroll
                for (int e = q * GQ; e < q * GQ + GQ; ++e) f(y[e], e < lim);
            }
        }
    };
    const int nfull = w / BL, rem = w - nfull * BL;
    uint32_t ya[BL], yb[BL];
    load(ya, 0);
    int b = 0;
    for (; b + 2 <= nfull; b += 2) {
        load_full(yb, (b + 1) * BL);
        use(ya, BL);
        load(ya, (b + 2) * BL);
        use(yb, BL);
    }
    if (b < nfull) {
        load(yb, (b + 1) * BL);
        use(ya, BL);
        if (rem) use(yb, rem);
    } else if (rem) {
        use(ya, rem);
    }
    const uint32_t *bk = (const uint32_t *)bv;
    int c = 0;
    for (; c + BL <= w; c += BL) {
        uint32_t y[BL];
#pragma unroll
        for (int e = 0; e < BL; ++e) y[e] = bk[c + e];
        use(y, BL);
    }
    if (c < w) {
        uint32_t y[BL];
        const int lim = w - c;
#pragma unroll
        for (int q = 0; q < BL / GQ; ++q) {
            if (q * GQ < lim) {
#pragma unroll
                for (int e = q * GQ; e < q * GQ + GQ; ++e) y[e] = bk[min(c + e, wm1)];
            }
        }
        use(y, lim);
    }
}

// Per-thread list of bracket keys at L[x * NS], x <= CAP (NS: threads of the
// workgroup).  Every key is stored at slot min(nl, CAP); nl advances only for
// keys inside [lo, lo + span], so slots 0 .. nl-1 end up holding exactly those
// (no branches, no selects).
template <int NS>
struct Bracket {
    uint32_t lo, span;
    int below, nl;
    uint32_t *L;
    // An invalid key becomes 0xFFFFFFFF, which is neither below lo nor inside
    // (span < 2^31).  Four VALU operations count it: the borrow of key - lo
    // is carried into below, the range test into nl.
    __device__ __forceinline__ void operator()(uint32_t key, bool valid) {
        key = valid ? key : 0xFFFFFFFFu;
        L[min(nl, CAP) * NS] = key;
        uint32_t d;
        asm("v_sub_co_u32_e32 %0, vcc, %2, %3\n\t"
            "v_addc_co_u32_e32 %1, vcc, 0, %1, vcc"
            : "=v"(d), "+v"(below)
            : "v"(key), "v"(lo)
            : "vcc");
        asm("v_cmp_le_u32_e32 vcc, %1, %2\n\t"
            "v_addc_co_u32_e32 %0, vcc, 0, %0, vcc"
            : "+v"(nl)
            : "v"(d), "v"(span)
            : "vcc");
    }
};

// Per-thread radix select of the key range [lo, hi) holding ranks r1 .. r2
// (1-based) of one window's 2w values.  Histograms live in the thread's list
// slots (bucket NB takes the keys outside the range).  A thread stops when its
// range holds at most CAP values or one key; the wave stops once at most two
// threads are left (a full pass costs the whole wave; those threads' brackets
// overflow and the wave's cooperative select finishes them).
template <int NS>
__device__ __forceinline__ void lane_band(__amdgpu_buffer_rsrc_t R, uint32_t voff, uint32_t rstr, const float *bv,
                                          int w, int k, int r1, int r2, uint32_t *H, uint32_t &lo_out,
                                          uint32_t &hi_out) {
    uint32_t lo = 0u, hi = 0x7F800000u;
    int base = 0, shift = -1;
    bool done = false;
    for (int level = 0; level < 16; ++level) {
        if (__popcll(__ballot(!done)) <= (level > 0 ? 2 : 0)) break;
#pragma unroll
        for (int b = 0; b <= NB; ++b) H[b * NS] = 0u;
        // level 0 buckets by pairs of binades, 2^-31 .. 2^1 (bucket b holds
        // exponents 96+2b and 97+2b; the end buckets take the rest); later
        // levels split [lo, hi) into NB equal key ranges
        const bool l0 = level == 0;
        const int sh = l0 ? 24 : max(shift, 0);
        const uint32_t kb = l0 ? 48u << 24 : lo;
        const uint32_t span = hi - lo;
        window_pass(R, voff, rstr, bv, w, [&](uint32_t key, bool valid) {
            int b = min(max((int)(key - kb) >> sh, 0), NB - 1);
            b = (valid && key - lo < span) ? b : NB;                    // lo <= key < hi
            __hip_atomic_fetch_add(H + b * NS, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
        });
        int acc = base, b1 = -1, b2 = NB - 1, below1 = base;
        bool fb2 = false;
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int cb = (int)H[b * NS];
            if (b1 < 0 && acc + cb >= r1) {
                b1 = b;
                below1 = acc;
            }
            if (!fb2 && acc + cb >= r2) {
                b2 = b;
                fb2 = true;
            }
            if (!fb2 || b == b2) acc += cb;
        }
        if (b1 < 0) b1 = b2;
        const int cnt = acc - below1;
        uint32_t nlo, nhi;
        if (l0) {
            nlo = b1 == 0 ? 0u : (uint32_t)(2 * b1 + 96) << 23;
            nhi = b2 == NB - 1 ? 0x7F800000u : (uint32_t)(2 * b2 + 98) << 23;
        } else {
            nlo = lo + ((uint32_t)b1 << sh);
            const uint64_t e = (uint64_t)lo + ((uint64_t)(b2 + 1) << sh);
            nhi = (uint32_t)(e < (uint64_t)hi ? e : (uint64_t)hi);
        }
        if (!done) {
            const bool stuck = (nlo == lo && nhi == hi);
            lo = nlo;
            hi = nhi;
            base = below1;
            if (hi - lo == 1u || cnt <= CAP) {
                done = true;
            } else {
                if (stuck) {  // the band spans the whole range: narrow to rank k alone
                    r1 = k;
                    r2 = k;
                }
                shift = max(0, (32 - __clz((int)(hi - lo - 1u))) - 4);
            }
        }
    }
    lo_out = lo;
    hi_out = hi;
}

// Workgroup barrier that orders LDS accesses only: global stores issued
// before it may still be in flight (nothing reads them before a full barrier).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Orders LDS accesses of the lanes of one wave (they execute in lockstep).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Per-wave LDS scratch of the cooperative select.
struct Coop {
    unsigned *hist;   // NB counters
    unsigned *cnt;    // 1 counter
    uint32_t *list;   // CAP keys
    uint32_t *sorted; // CAP keys
};
constexpr int COOP_FLOATS = NB + 4 + 2 * CAP;

// Exact ranks r1 .. r2 (1-based) of one window's 2w values for w <= 64, by
// the 64 lanes of a wave together: lane x holds A(x) = ab[x * gs] and B(x) =
// bv[x] and counts, for both, the values smaller than it, ties by position
// (the A values first, in row order, then the B values in column order); the
// other lanes' values come from their registers.  The values of ranks r1 ..
// r2 land in C.sorted in order; *below = r1 - 1.  A few hundred instructions,
// where the radix select takes several rounds of histograms.  Must be called
// by all lanes of the wave.
__device__ __forceinline__ int coop_rank(const float *ab, int gs, const float *bv, int w, int r1, int r2,
                                         const Coop &C, int lane, int *below) {
    const bool in = lane < w;
    const uint32_t a = in ? key_of(ab[(size_t)lane * gs]) : 0xFFFFFFFFu;  // outside: never counted
    const uint32_t b = in ? ((const uint32_t *)bv)[lane] : 0xFFFFFFFFu;
    int ra = 0, rb = 0;
    // valid keys are at most 0x7F800000, so key + 1 does not wrap
#pragma unroll 2
    for (int src = 0; src < w; ++src) {
        const uint32_t va = (uint32_t)__builtin_amdgcn_readlane((int)a, src);
        const uint32_t vb = (uint32_t)__builtin_amdgcn_readlane((int)b, src);
        const uint32_t lower = src < lane;
        ra += (va < a + lower) + (vb < a);   // A(src) before A(lane); every B after
        rb += (va <= b) + (vb < b + lower);  // every A before B(lane); B(src) before it
    }
    if (in && ra >= r1 - 1 && ra <= r2 - 1) C.sorted[ra - r1 + 1] = a;
    if (in && rb >= r1 - 1 && rb <= r2 - 1) C.sorted[rb - r1 + 1] = b;
    wave_sync();
    *below = r1 - 1;
    return r2 - r1 + 1;
}

// Exact radix select, by the 64 lanes of a wave together, of the key range
// holding ranks r1 .. r2 (1-based) of one window's 2w values: A(i) =
// ab[i * gs] for i < w and B(c) = bv[c] for c < w.  The
// search starts from the key range [lo, hi) that holds rank k, with `base`
// values below it (what the window's failed bracket pass established).  Every
// lane gets *below (values under the band found) and the count of values in
// it; those keys are left sorted in C.sorted.  If the band cannot be narrowed
// to CAP values the ranks shrink to k .. k.  Each lane keeps its share of the
// row minima (at most CW values) in registers; the column minima are in LDS.
// Must be called by all lanes of the wave.
constexpr int CW = (kMaxW + 63) / 64;
__device__ __forceinline__ int coop_band(const float *ab, int gs, const float *bv, int w, int k, int r1, int r2,
                                         uint32_t lo, uint32_t hi, int base, const Coop &C, int lane,
                                         int *below) {
    uint32_t ka[CW];
    const uint32_t *bk = (const uint32_t *)bv;
    const int nj = (w + 63) >> 6;
#pragma unroll
    for (int j = 0; j < CW; ++j) {
        ka[j] = 0xFFFFFFFFu;  // outside every range
        if (j < nj) {
            const int i = lane + 64 * j;
            if (i < w) ka[j] = key_of(ab[(size_t)i * gs]);
        }
    }
    for (int level = 0; level < 16; ++level) {
        const uint32_t span = hi - lo;
        const int shift = max(0, (32 - __clz((int)(span - 1u))) - 4);
        if (lane < NB) C.hist[lane] = 0u;
        wave_sync();
#pragma unroll
        for (int j = 0; j < CW; ++j) {
            if (j < nj) {
                if (ka[j] - lo < span) atomicAdd(&C.hist[(ka[j] - lo) >> shift], 1u);
            }
        }
        for (int c = lane; c < w; c += 64) {
            const uint32_t kc = bk[c];
            if (kc - lo < span) atomicAdd(&C.hist[(kc - lo) >> shift], 1u);
        }
        wave_sync();
        int acc = base, b1 = -1, b2 = NB - 1, below1 = base;
        for (int b = 0; b < NB; ++b) {
            const int cb = (int)C.hist[b];
            if (b1 < 0 && acc + cb >= r1) {
                b1 = b;
                below1 = acc;
            }
            if (acc + cb >= r2) {
                b2 = b;
                acc += cb;
                break;
            }
            acc += cb;
        }
        if (b1 < 0) b1 = b2;
        const int cnt = acc - below1;  // values in buckets b1 .. b2
        const uint32_t nlo = lo + ((uint32_t)b1 << shift);
        const uint64_t e = (uint64_t)lo + ((uint64_t)(b2 + 1) << shift);
        const uint32_t nhi = (uint32_t)(e < (uint64_t)hi ? e : (uint64_t)hi);
        const bool stuck = (nlo == lo && nhi == hi);
        lo = nlo;
        hi = nhi;
        base = below1;
        wave_sync();  // every lane has read the histogram
        if (hi - lo == 1u) {  // one key value holds ranks r1 .. r2
            if (lane == 0) C.sorted[0] = lo;
            wave_sync();
            *below = base;
            return 1;
        }
        if (cnt <= CAP) {
            if (lane == 0) *C.cnt = 0u;
            wave_sync();
            const uint32_t sp = hi - lo;
#pragma unroll
            for (int j = 0; j < CW; ++j) {
                if (j < nj) {
                    if (ka[j] - lo < sp) C.list[atomicAdd(C.cnt, 1u)] = ka[j];
                }
            }
            for (int c = lane; c < w; c += 64) {
                const uint32_t kc = bk[c];
                if (kc - lo < sp) C.list[atomicAdd(C.cnt, 1u)] = kc;
            }
            wave_sync();
            if (lane < cnt) {  // rank of each key, ties by position
                const uint32_t y = C.list[lane];
                int r = 0;
                for (int x = 0; x < cnt; ++x) {
                    const uint32_t yx = C.list[x];
                    r += (yx < y) || (yx == y && x < lane);
                }
                C.sorted[r] = y;
            }
            wave_sync();
            *below = base;
            return cnt;
        }
        if (stuck) {  // the band spans the whole range: narrow to rank k alone
            r1 = k;
            r2 = k;
        }
    }
    *below = base;  // not reached for finite keys
    if (lane == 0) C.sorted[0] = lo;
    wave_sync();
    return 1;
}

// Global-to-LDS copy of n doubles by NT threads, four loads in flight per
// thread before their stores.
template <int NT>
__device__ __forceinline__ void stage_f64(double *dst, const double *src, int n, int t) {
    constexpr int U = 4;
    for (int b = t; b < n; b += U * NT) {
        double v[U];
#pragma unroll
        for (int e = 0; e < U; ++e) v[e] = b + e * NT < n ? src[b + e * NT] : 0.0;
#pragma unroll
        for (int e = 0; e < U; ++e)
            if (b + e * NT < n) dst[b + e * NT] = v[e];
    }
}

// Centred covariance of row r = rb + i and column C0 + u by a direct FP64 dot
// product (the anchor of a diagonal).
__device__ __forceinline__ float anchor_at(const ProfileJob &J, int64_t rb, int i, int64_t C0, int u) {
    const double *xr = J.row.xc + rb + i;
    const double *xcp = J.col.xc + C0 + u;
    double acc = 0.0;
    for (int tt = 0; tt < J.l; ++tt) acc = fma(xr[tt], xcp[tt], acc);
    return (float)(acc - (double)J.l * J.row.mu[rb + i] * J.col.mu[C0 + u]);
}

// FP64 anchors (centred covariance at the first cell) of a thread's V
// diagonals d0 .. d0+V-1 of a sub-tile: xr[q] is the centred series at the
// query's row q, xc[q] at column q of the sub-tile (LDS or global memory).
// A thread's diagonals either all start in row 0 (ub0 = d0-(w-1) >= 0, first
// cell (0, ub0+v)) or all start in column 0 (first cell (w-1-d0-v, 0)); both
// are the sums acc[j] = sum_t P[t] Q[t+j], j < V, register-blocked along t:
// P = xr, Q = xc + ub0 for the first kind, P = xc, Q = xr + w-1-d0-(V-1) (and
// j = V-1-v) for the second.  Diagonals d < 0 or d >= ndg get 0.
template <int V>
__device__ __forceinline__ void diag_anchors(float (&cov)[V], const double *xr, const double *xc, bool act,
                                             int d0, int w, int l, int ndg, const double *mur, const double *muc) {
#pragma unroll
    for (int v = 0; v < V; ++v) cov[v] = 0.0f;
    if (!act) return;
    const int ub0 = d0 - (w - 1);
    const bool top = ub0 >= 0;
    const int base = -ub0 - (V - 1);
    const double *P = top ? xr : xc;
    const double *Q = top ? xc + ub0 : xr + base;
    double acc[V], xs[V];
#pragma unroll
    for (int v = 0; v < V; ++v) acc[v] = 0.0;
#pragma unroll
    for (int v = 0; v < V - 1; ++v) xs[v] = Q[v];
    int tt = 0;
    for (; tt + V <= l; tt += V) {
#pragma unroll
        for (int kq = 0; kq < V; ++kq) {
            xs[(kq + V - 1) % V] = Q[tt + kq + V - 1];
            const double a = P[tt + kq];
#pragma unroll
            for (int v = 0; v < V; ++v) acc[v] = fma(a, xs[(kq + v) % V], acc[v]);
        }
    }
    for (; tt < l; ++tt) {
        const double a = P[tt];
#pragma unroll
        for (int v = 0; v < V; ++v) acc[v] = fma(a, Q[tt + v], acc[v]);
    }
#pragma unroll
    for (int v = 0; v < V; ++v) {
        const int d = d0 + v;
        const double c = top ? acc[v] - (double)l * mur[0] * muc[ub0 + v]
                             : acc[V - 1 - v] - (double)l * mur[base + V - 1 - v] * muc[0];
        if (d >= 0 && d < ndg) cov[v] = (float)c;
    }
}

// LDS carve of one tile.  Distance phase: packed row statistics, packed
// column statistics and column minima of the sub-tile, per-wave block minima,
// RCH rows of y.  Each row of y has w-1 columns of margin before column 0 and
// w+V after the sub-tile, where the cells of the partial diagonals that lie
// outside the sub-tile land.  Selection phase (same memory): column minima of
// the tile, per-thread lists, per-wave scratch of the cooperative select.
struct Carve {
    float4 *rst;   // rows: {inv/2, df, dg, h/2}
    float4 *cst;   // cst[u + 1] for column u, -1 <= u <= CS+V: {inv, df, dg, (1-h)/2}; zeros outside
    float *colS, *BMv, *buf;
    int ldb, lm;   // row stride of buf; margin before column 0 (w-1, plus V-1 for
                   // the diagonals d < 0 of the first thread)
    float *colY, *lst, *coop;
    __device__ Carve(float *sm, int NT, int w, int V, int RCH, int CWS, int CWT) {
        const int w4 = (w + 3) & ~3;
        const int c4 = (CWS + 8 + 3) & ~3;
        rst = (float4 *)sm;
        cst = rst + w4;
        colS = (float *)(cst + c4);
        BMv = colS + c4;
        buf = BMv + RCH * BMW;
        lm = w - 1 + V - 1;
        ldb = (lm + CWS + w + V + 3) & ~3;
        colY = sm;
        lst = colY + ((CWT + 3) & ~3);
        coop = lst + (CAP + 1) * NT;
    }
};

template <int NT, int V, int RCH>
__global__ void __launch_bounds__(NT, 2) k_profile(ProfileArgs A) {
    constexpr int NW = NT / 64;                    // waves
    constexpr int RPW = RCH > NW ? RCH / NW : 1;   // rows per wave in the row-minimum step
    constexpr int LPR = 64 / RPW;                  // lanes (blocks) per row
    extern __shared__ __align__(16) float sm[];
    __shared__ uint32_t next_tile;
    const Geo g = A.g;
    const int JT = g.JT, nA = g.nA, SBW = g.SBW;
    const int t = threadIdx.x;
    const int wv = t >> 6, lane = t & 63;
    const int64_t total = A.B.tile_end[A.B.njobs - 1];
    int64_t gt = blockIdx.x;
    if (A.B.counter) {  // tiles handed out by a device work counter
        if (t == 0) next_tile = atomicAdd(A.B.counter, 1u);
        __syncthreads();
        gt = next_tile;
    }
    while (gt < total) {
        int jb = 0;
        while (jb + 1 < A.B.njobs && gt >= A.B.tile_end[jb]) ++jb;
        const ProfileJob &J = A.B.J[jb];
        const int64_t tile = gt - (jb > 0 ? A.B.tile_end[jb - 1] : 0);
        const int w = J.w, l = J.l;
        const int64_t ntile = (J.Nm + JT - 1) / JT;
        const int keff = min(J.k, 2 * w);
        const int pstr = w * nA;              // scratch floats per window-in-block
        const int CWT = JT + w - 1;           // columns of a tile
        const int CWS = SBW + w - 1;          // columns of a sub-tile
        const float four_l = (float)(4 * l);
        const Carve M(sm, NT, w, V, RCH, CWS, CWT);

        float *rw = J.rw + (size_t)blockIdx.x * A.B.slot_floats;   // row minima of the tile
        float *colG = rw + (size_t)pstr * G;                      // column minima of the tile
        const __amdgpu_buffer_rsrc_t R =
            __builtin_amdgcn_make_buffer_rsrc(rw, (short)0, (int)(A.B.slot_floats * 4), 0x00020000);
        float tmax = 0.0f;

        const int s = (int)(tile / ntile);
        const int64_t J0 = (tile % ntile) * JT;
        const int JTe = (int)min<int64_t>(JT, J.Nm - J0);
        const int64_t rb = (int64_t)s * J.row_stride;

        __syncthreads();  // the previous tile is done with LDS and the scratch slot
        PROBE_MARK(tDist);
        int crow = 0;     // a constant row (h != 0) takes the general path
        for (int i = t; i < w; i += NT) {
            // y = (0.5 - h_r/2 - h_c/2) - cov * (inv_r/2) * inv_c: constant
            // windows (h = 0.5, inv = 0) follow the conventions of the stats
            const int64_t r = rb + i;
            const float hr = J.row.h[r];
            M.rst[i] = make_float4(0.5f * J.row.inv[r], J.row.df[r], J.row.dg[r], 0.5f * hr);
            crow |= hr != 0.0f;
        }
        const bool any_const = __syncthreads_or(crow) != 0;
        // re-anchoring at chunk starts keeps the fast path
        const bool anchor_chunks = J.anchor_every > 0 && J.anchor_every % RCH == 0;
        const bool fast_tile = !any_const && (J.anchor_every == 0 || anchor_chunks);

        for (int Js = 0; Js < JTe; Js += SBW) {
            const int JSe = min(SBW, JTe - Js);   // windows of this sub-tile
            const int CS = JSe + w - 1;           // its columns
            const int nbl = (CS + G - 1) / G;     // blocks of G columns
            const bool last = Js + SBW >= JTe;
            const int own = last ? CS : SBW;      // columns whose minima it owns
            const int64_t C0 = J0 + Js;           // first column (series index)
            const int ldb = M.ldb;
            lds_barrier();  // previous sub-tile done with the shared region
            {
                // entry u holds column u-1; columns -1 and CS+V (and all past
                // them, by clamping) read as zeros: df = dg = 0 there, so a
                // partial diagonal's covariance stays at its anchor until the
                // diagonal enters the sub-tile.  All of a thread's loads are
                // issued before its stores (CS + V + 2 <= kStageIters * NT).
                float4 cv[kStageIters];
#pragma unroll
                for (int it = 0; it < kStageIters; ++it) {
                    const int u = t + it * NT;
                    float4 c = make_float4(0.0f, 0.0f, 0.0f, 0.5f);
                    if (u >= 1 && u <= CS + V) {
                        const int64_t cc = C0 + u - 1;
                        c = make_float4(J.col.inv[cc], J.col.df[cc], J.col.dg[cc], 0.5f - 0.5f * J.col.h[cc]);
                    }
                    cv[it] = c;
                }
#pragma unroll
                for (int it = 0; it < kStageIters; ++it) {
                    const int u = t + it * NT;
                    if (u < CS + V + 2) M.cst[u] = cv[it];
                    if (u < CS) M.colS[u] = INFINITY;
                }
            }

            // Thread t owns diagonals t*V-off .. t*V-off+V-1, diagonal d the
            // cells (i, u = d - (w-1) + i); off makes w-1 a multiple of V, so
            // that no thread holds diagonals of both the lower triangle
            // (d < w-1) and the rest.  Every thread runs every row; the cells
            // of a partial diagonal outside 0 <= u < CS, and all cells of the
            // diagonals d < 0, go to the row margins and are never read.
            const int ndg = CS + w - 1;             // diagonals of the sub-tile
            const int off = (V - (w - 1) % V) % V;
            const int nT = (ndg + off + V - 1) / V; // threads with diagonals
            const bool act = t < nT;
            const int d0 = t * V - off;
            const int ub0 = d0 - (w - 1);

            PROBE_MARK(tAnc);
            // 1. FP64 anchors.  The sub-tile's slice of the centred series
            //    (columns 0 .. CS+V+l-1, the query's rows 0 .. w+l+V-3) is
            //    staged in the row buffer, free until the first chunk, when it
            //    fits.
            const int ncx = CS + V + l;
            const int nrx = w + l + V - 2;
            const bool staged = 2 * (ncx + nrx) <= RCH * ldb;
            float cov[V];
            if (staged) {
                double *Xc = (double *)M.buf, *Xr = Xc + ncx;
                stage_f64<NT>(Xc, J.col.xc + C0, ncx, t);
                stage_f64<NT>(Xr, J.row.xc + rb, nrx, t);
                lds_barrier();
                diag_anchors<V>(cov, Xr, Xc, act, d0, w, l, ndg, J.row.mu + rb, J.col.mu + C0);
            } else {
                diag_anchors<V>(cov, J.row.xc + rb, J.col.xc + C0, act, d0, w, l, ndg, J.row.mu + rb,
                                J.col.mu + C0);
            }
            lds_barrier();
            PROBE_SPAN(17, tAnc);

            // register window of column statistics: slot (v + k) % V holds the
            // column of diagonal v at row k of the current chunk; row k loads
            // the column of diagonal V-1 into slot (k + V - 1) % V
            const int cmax = CS + V + 1;
            float wi[V], wf[V], wg[V], wa[V];
#pragma unroll
            for (int v = 0; v < V - 1; ++v) {
                const float4 c = M.cst[min(max(ub0 + v + 1, 0), cmax)];
                wi[v] = c.x;
                wf[v] = c.y;
                wg[v] = c.z;
                wa[v] = c.w;
            }

            for (int R0 = 0; R0 < w; R0 += RCH) {
                const int nr = min(RCH, w - R0);
                // 2. rows R0 .. R0+nr-1 of y into buf
                PROBE_MARK(tRec);
                const bool fast = fast_tile && R0 + RCH <= w;
                if (act) {
                    if (fast && anchor_chunks && R0 > 0 && R0 % J.anchor_every == 0) {
                        // FP64 re-anchor at the chunk start: the FP32 recurrence
                        // never runs more than anchor_every steps
#pragma unroll
                        for (int v = 0; v < V; ++v) {
                            const int u = ub0 + v + R0;
                            if (u >= 0 && u < CS) cov[v] = anchor_at(J, rb, R0, C0, u);
                        }
                    }
                    if (fast) {
                        // all rows present, no constant rows: no branches; the
                        // chunk's statistics are loaded ahead of its LDS stores
                        float4 cc[RCH], rr4[RCH];
#pragma unroll
                        for (int k = 0; k < RCH; ++k) {
                            cc[k] = M.cst[min(max(ub0 + V + R0 + k, 0), cmax)];
                            rr4[k] = M.rst[R0 + k];
                        }
#pragma unroll
                        for (int k = 0; k < RCH; ++k) {
                            const int i = R0 + k;
                            const int sl = (k + V - 1) % V;
                            wi[sl] = cc[k].x;
                            wf[sl] = cc[k].y;
                            wg[sl] = cc[k].z;
                            wa[sl] = cc[k].w;
                            const float4 r = rr4[k];
                            float *brow = M.buf + k * ldb + M.lm + ub0 + i;
#pragma unroll
                            for (int v = 0; v < V; ++v) {
                                const int s2 = (v + k) % V;
                                brow[v] = __builtin_amdgcn_fmed3f(fmaf(-cov[v] * r.x, wi[s2], wa[s2]), 0.0f, 1.0f);
                                cov[v] = fmaf(r.y, wg[s2], fmaf(wf[s2], r.z, cov[v]));
                            }
                        }
                    } else {
#pragma unroll
                        for (int k = 0; k < RCH; ++k) {
                            const int i = R0 + k;
                            if (i < w) {
                                const int sl = (k + V - 1) % V;
                                const float4 c = M.cst[min(max(ub0 + V + i, 0), cmax)];
                                wi[sl] = c.x;
                                wf[sl] = c.y;
                                wg[sl] = c.z;
                                wa[sl] = c.w;
                                if (J.anchor_every > 0 && i > 0 && i % J.anchor_every == 0) {
#pragma unroll
                                    for (int v = 0; v < V; ++v) {
                                        const int u = ub0 + v + i;
                                        if (u >= 0 && u < CS) cov[v] = anchor_at(J, rb, i, C0, u);
                                    }
                                }
                                const float4 r = M.rst[i];
                                float *brow = M.buf + k * ldb + M.lm + ub0 + i;
#pragma unroll
                                for (int v = 0; v < V; ++v) {
                                    const int s2 = (v + k) % V;
                                    brow[v] = __builtin_amdgcn_fmed3f(fmaf(-cov[v] * r.x, wi[s2], wa[s2] - r.w),
                                                                      0.0f, 1.0f);
                                    cov[v] = fmaf(r.y, wg[s2], fmaf(wf[s2], r.z, cov[v]));
                                }
                            }
                        }
                    }
                    // the next chunk starts at k = 0: slot v must hold what
                    // slot (v + RCH) % V holds now
                    float ti[V], tf[V], tg[V], ta[V];
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        ti[v] = wi[(v + RCH) % V];
                        tf[v] = wf[(v + RCH) % V];
                        tg[v] = wg[(v + RCH) % V];
                        ta[v] = wa[(v + RCH) % V];
                    }
#pragma unroll
                    for (int v = 0; v < V; ++v) {
                        wi[v] = ti[v];
                        wf[v] = tf[v];
                        wg[v] = tg[v];
                        wa[v] = ta[v];
                    }
                }
                lds_barrier();
                PROBE_SPAN(18, tRec);
                PROBE_MARK(tCol);
                // 3. column minima of y (eq. 10) for the columns this sub-tile owns
                if (nr == RCH) {
                    for (int u = t; u < own; u += NT) {
                        const float *col = M.buf + M.lm + u;
                        float m[RCH];
#pragma unroll
                        for (int rr = 0; rr < RCH; ++rr) m[rr] = col[rr * ldb];
                        float mn = M.colS[u];
#pragma unroll
                        for (int rr = 0; rr < RCH; ++rr) mn = umin(mn, m[rr]);
                        M.colS[u] = mn;
                    }
                } else {
                    for (int u = t; u < own; u += NT) {
                        float mn = M.colS[u];
                        for (int rr = 0; rr < nr; ++rr) mn = umin(mn, M.buf[rr * ldb + M.lm + u]);
                        M.colS[u] = mn;
                    }
                }
                PROBE_SPAN(19, tCol);
                PROBE_MARK(tRow);
                // 4. sliding row minima of width w (eq. 11): each wave takes
                //    RPW rows of the chunk, LPR lanes per row; lane al takes
                //    the windows of block al of the sub-tile.  Columns past CS
                //    only reach windows past the sub-tile's last.
                const int rr = wv * RPW + lane / LPR;
                if (rr < nr) {
                    const float *row = M.buf + rr * ldb + M.lm;
                    float *BM = M.BMv + rr * BMW;
                    const int al = lane % LPR;
                    float S[G];
                    {
                        // lanes past the last block repeat it (never read back)
                        const float *src = row + min(al, nbl - 1) * G;
#pragma unroll
                        for (int j = 0; j < G; ++j) S[j] = src[j];
#pragma unroll
                        for (int j = G - 2; j >= 0; --j) S[j] = umin(S[j], S[j + 1]);
                    }
                    BM[al] = S[0];
                    if (al + LPR < nbl) {  // blocks past the lanes: their minima only
                        const float *src = row + (al + LPR) * G;
                        float X[G];
#pragma unroll
                        for (int j = 0; j < G; ++j) X[j] = src[j];
                        float mn = X[0];
#pragma unroll
                        for (int j = 1; j < G; ++j) mn = umin(mn, X[j]);
                        BM[al + LPR] = mn;
                    }
                    wave_sync();
                    if (al * G < JSe) {
                        const int a = Js / G + al;   // block inside the tile
                        // scratch layout: row i of window p of block a at
                        // (p * w + i) * nA + a
                        const uint32_t vo = (uint32_t)((R0 + rr) * nA + a) * 4u;
                        if (w <= G) {
                            for (int p = 0; p < G; ++p) {
                                const int v = al * G + p;
                                float mn = row[v];
                                for (int c = 1; c < w; ++c) mn = umin(mn, row[v + c]);
                                __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(mn), R, (int)vo,
                                                                      (int)((uint32_t)(p * pstr) * 4u), 0);
                            }
                        } else {
                            // window p: columns al*G + p .. al*G + p + w - 1 =
                            // suffix of block al, blocks al+1 .. al+q-1, and the
                            // columns (al+q)*G .. al*G + w - 1 + p
                            const int q = (w - 1) / G;
                            const int rp = (w - 1) - q * G;
                            // the tail columns, loaded ahead of the stores below
                            const float *tl = row + al * G + w - 1;
                            float T[G];
#pragma unroll
                            for (int p = 1; p < G; ++p) T[p] = tl[p];
                            float base = INFINITY;
#pragma unroll 4
                            for (int b = al + 1; b < al + q; ++b) base = umin(base, BM[b]);
                            const float *pb = row + (al + q) * G;
#pragma unroll 4
                            for (int x = 0; x <= rp; ++x) base = umin(base, pb[x]);
                            float pr = base;
#pragma unroll
                            for (int p = 0; p < G; ++p) {
                                if (p > 0) pr = umin(pr, T[p]);
                                __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(umin(S[p], pr)), R, (int)vo,
                                                                      (int)((uint32_t)(p * pstr) * 4u), 0);
                            }
                        }
                    }
                }
                lds_barrier();
                PROBE_SPAN(20, tRow);
            }
            // column minima of the owned columns to the tile's copy
            for (int u = t; u < own; u += NT) colG[Js + u] = M.colS[u];
        }

        // 5. selection (eqs. 12-13): k-th smallest y of the w row minima and the
        //    w column minima of each window; thread a takes block a in order.
        //    Windows whose bracket misses are solved by the whole wave together.
        __syncthreads();  // the distance phase is done with LDS; colG is written
        PROBE_SPAN(16, tDist);
        PROBE_MARK(tSel);
        float *colY = M.colY;
        for (int u0 = t; u0 < CWT; u0 += 8 * NT) {  // eight loads in flight per thread
            float cy[8];
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int u = u0 + e * NT;
                cy[e] = u < JTe + w - 1 ? colG[u] : INFINITY;
            }
#pragma unroll
            for (int e = 0; e < 8; ++e)
                if (u0 + e * NT < CWT) colY[u0 + e * NT] = cy[e];
        }
        lds_barrier();
        if (t < nA && (t & ~63) * G < JTe) {  // waves with a window in the tile
            uint32_t *L = (uint32_t *)M.lst + t;
            float *cs = M.coop + wv * COOP_FLOATS;
            const Coop C{(unsigned *)cs, (unsigned *)(cs + NB), (uint32_t *)(cs + NB + 4),
                         (uint32_t *)(cs + NB + 4 + CAP)};
            const int r1 = max(1, keff - BAND), r2 = min(2 * w, keff + BAND);
            uint32_t blo = 0u, bhi = 0u, ystar = 0u;
            const uint32_t rstr = (uint32_t)nA * 4u;  // bytes between rows
            for (int p = 0; p < G; ++p) {
                const int v = t * G + p;
                const bool valid = v < JTe;
                const uint32_t voff = (uint32_t)(p * pstr + t) * 4u;
                PROBE(0, valid);
                PROBE_MARK(tRun);
                if (p == 0) {  // run start: the bracket from a radix select
                    uint32_t klo, khi;
                    PROBE(1, valid);
                    lane_band<NT>(R, voff, rstr, colY + v, w, keff, r1, r2, L, klo, khi);
                    blo = klo;
                    bhi = khi - 1u;
                }
                PROBE_SPAN(22, tRun);
                PROBE_MARK(tPass);
                // Results of the last pass of this window: its bracket [plo,
                // phi], the values under it (pb) and in it (pn), the rank of
                // the k-th among those in it (pk); L holds them sorted.
                uint32_t plo = blo, phi = bhi;
                int pb, pn, pk;
                auto pass = [&](uint32_t lo, uint32_t hi) {
                    Bracket<NT> Bk{lo, hi - lo, 0, 0, L};
                    window_pass(R, voff, rstr, colY + v, w, Bk);
                    plo = lo;
                    phi = hi;
                    pb = Bk.below;
                    pn = Bk.nl;
                    pk = keff - pb;
                    uint32_t srt[CAP];
#pragma unroll
                    for (int x = 0; x < CAP; ++x) srt[x] = x < pn ? L[x * NT] : 0xFFFFFFFFu;
                    sort_net(srt);
#pragma unroll
                    for (int x = 0; x < CAP; ++x) L[x * NT] = srt[x];
                };
                // the pass held rank k: in its list, or, for a bracket of one
                // key, in a list that overflowed (every value in it is that key)
                auto held = [&]() { return pk >= 1 && pk <= pn && (pn <= CAP || plo == phi); };
                // rank k, and the next bracket: ranks k-BAND .. k+BAND of this
                // window, or extrapolated from the list's spacing where it ends
                auto take = [&]() {
                    if (pn > CAP) {  // one-key bracket: keep it
                        ystar = plo;
                        blo = bhi = plo;
                        return;
                    }
                    ystar = L[(pk - 1) * NT];
                    const int q1 = r1 - pb, q2 = r2 - pb;
                    const float l0 = __uint_as_float(L[0]), l1 = __uint_as_float(L[(pn - 1) * NT]);
                    const float sp = (l1 - l0) / (float)max(pn - 1, 1);
                    blo = q1 >= 1 ? L[(q1 - 1) * NT] : key_of(fmaxf(l0 - 1.5f * (float)(1 - q1) * sp, 0.0f));
                    bhi = q2 <= pn ? L[(q2 - 1) * NT] : key_of(l1 + 1.5f * (float)(q2 - pn) * sp);
                };
                pass(blo, bhi);
                bool ok = held();
                PROBE_SPAN(23, tPass);
                PROBE_MARK(tSort);
                PROBE(2, valid && ok);
                PROBE(4, valid && !ok && pk < 1);
                PROBE(5, valid && !ok && pk > pn && pn <= CAP);
                PROBE(6, valid && pn > CAP);
                PROBE(7, valid && !ok && p == 0);
                PROBE(8, valid && pn > CAP && plo == phi);
                PROBE(9, valid ? pn : 0);
                PROBE(10, valid && pn > CAP && pk >= 1 && pk <= pn);
                if (ok) take();
                // A bracket that missed rank k gets one more pass, by all such
                // lanes of the wave at once (when there are RETRY_MIN of
                // them), with a bracket re-aimed at ranks
                // k-BAND .. k+BAND: under it, everything (when that is few
                // values) or the list's spacing extrapolated down from it;
                // over it, the spacing extrapolated up; inside an
                // overflowing list, the stretch of the list (a sample of the
                // bracket's values) around rank k's share.  A second miss
                // goes to the wave's cooperative select.
                // Lanes without a second pass repeat their first one (the
                // next window's bracket, or the same missed bracket), so that
                // a missed bracket's counts stay what the select starts from.
                // A bracket must satisfy lo <= hi: the pass relies on
                // hi - lo < 2^31.
                uint32_t rlo = blo, rhi = bhi;
                bool retry = false;
                if (valid && !ok) {
                    const int nk = min(pn, CAP);  // sorted values in L
                    const float l0 = __uint_as_float(L[0]), l1 = __uint_as_float(L[(max(nk, 1) - 1) * NT]);
                    // spacing of the values near the bracket: the list's, or
                    // the bracket's width over the band where the list is short
                    const float sp = nk >= 2 && l1 > l0
                                         ? (l1 - l0) / (float)(nk - 1)
                                         : (__uint_as_float(phi) - __uint_as_float(plo)) / (float)(2 * BAND);
                    uint32_t tlo = 1u, thi = 0u;
                    if (pn > CAP) {  // overflow around rank k: the list is a sample of the bracket
                        if (pk >= 1 && pk <= pn) {
                            const int q = (pk - 1) * CAP / pn, d = max(1, (BAND + 2) * CAP / pn);
                            tlo = q - d <= 0 ? plo : L[(q - d) * NT];
                            thi = q + d >= CAP - 1 ? phi : L[(q + d) * NT];
                        }
                    } else if (pk < 1) {  // rank k under the bracket, pb values there
                        const bool all = pb <= CAP && r2 <= CAP;
                        if (all || sp > 0.0f) {
                            tlo = all ? 0u
                                      : key_of(fmaxf(__uint_as_float(plo) - 1.5f * (float)(pb - r1 + 2) * sp, 0.0f));
                            thi = r2 <= pb ? plo - 1u : (r2 - pb <= pn ? L[(r2 - pb - 1) * NT] : phi);
                        }
                    } else if (sp > 0.0f) {  // rank k over the bracket
                        tlo = r1 <= pb ? plo : (r1 - pb <= pn ? L[(r1 - pb - 1) * NT] : phi + 1u);
                        thi = key_of(__uint_as_float(phi) + 1.5f * (float)(r2 - pb - pn + 1) * sp);
                    }
                    if (tlo <= thi) {
                        rlo = tlo;
                        rhi = thi;
                        retry = true;
                    }
                }
                PROBE(11, retry);
                if (__popcll(__ballot(retry)) >= RETRY_MIN) {
                    pass(rlo, rhi);
                    if (retry && held()) {
                        ok = true;
                        take();
                    }
                    PROBE(12, retry && ok);
                }
                // where the k-th value lies, from the last pass: below its
                // bracket, above it, or inside an overflowing list
                uint32_t flo = 0u, fhi = phi + 1u;
                int fbase = 0;
                if (pk > pn) {
                    flo = phi + 1u;
                    fhi = 0x7F800000u;
                    fbase = pb + pn;
                } else if (pk >= 1) {
                    flo = plo;
                    fbase = pb;
                } else {
                    fhi = plo;
                }
                PROBE_SPAN(24, tSort);
                PROBE_MARK(tCoop);
                uint64_t need = __ballot(valid && !ok);
                while (need) {
                    const int ln = __ffsll((unsigned long long)need) - 1;
                    need &= need - 1;
                    const int tf = (t & ~63) + ln;
                    int below = 0;
                    const uint32_t clo = (uint32_t)__shfl((int)flo, ln), chi = (uint32_t)__shfl((int)fhi, ln);
                    const int cbase = __shfl(fbase, ln);
                    // short windows: the band's ranks counted outright;
                    // longer ones: a radix select from the failed pass's range
                    const float *ab = rw + p * pstr + tf, *bw = colY + tf * G + p;
                    const bool by_rank = w <= 64;
                    const int nc = by_rank ? coop_rank(ab, nA, bw, w, r1, r2, C, lane, &below)
                                           : coop_band(ab, nA, bw, w, keff, r1, r2, clo, chi, cbase, C, lane,
                                                       &below);
                    if (lane == ln) {
                        PROBE(3, 1);
                        const int kk2 = keff - below;
                        ystar = C.sorted[min(max(kk2, 1), nc) - 1];
                        uint32_t nlo = C.sorted[min(max(r1 - below, 1), nc) - 1];
                        uint32_t nhi = C.sorted[min(max(r2 - below, 1), nc) - 1];
                        // The radix select searched only the side of the
                        // last bracket that holds rank k.  Ranks of the next
                        // bracket on the other side come from that pass (its
                        // sorted list, or the bracket's end), so that the next
                        // bracket spans ranks k-BAND .. k+BAND again instead of
                        // shrinking to the searched side.
                        if (!by_rank && pn <= CAP && pk < 1 && r2 > pb)
                            nhi = r2 - pb <= pn ? L[(r2 - pb - 1) * NT] : phi;
                        if (!by_rank && pn <= CAP && pk > pn && r1 <= pb + pn)
                            nlo = r1 > pb ? L[(r1 - pb - 1) * NT] : plo;
                        blo = nlo;
                        bhi = nhi;
                    }
                    wave_sync();
                }
                PROBE_SPAN(25, tCoop);
                if (valid) {
                    const float dist = sqrtf(four_l * __uint_as_float(ystar));
                    J.D[(int64_t)s * J.ld + J0 + v] = dist;
                    tmax = fmaxf(tmax, dist);
                }
            }
        }

        PROBE_SPAN(21, tSel);
        // max of D over this tile (the denominator of eq. 18): one atomic per wave
        if (J.dmax_bits) {
            float mx = tmax;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
            if (lane == 0) atomicMax(J.dmax_bits, __float_as_uint(mx));
        }
        if (A.B.counter) {
            __syncthreads();
            if (t == 0) next_tile = atomicAdd(A.B.counter, 1u);
            __syncthreads();
            gt = next_tile;
        } else {
            gt += gridDim.x;
        }
    }
}

constexpr int kCUs = 256;                 // compute units of an MI355X
constexpr size_t kLdsOne = 158 * 1024;    // LDS budget of one workgroup per CU
constexpr size_t kLdsTwo = 78 * 1024;     // per workgroup with two per CU

size_t lds_floats(int w, const Geo &g) {
    const size_t cwt4 = (((size_t)g.JT + w - 1) + 3) & ~(size_t)3;
    const size_t cws = (size_t)g.SBW + w - 1;
    const size_t c4 = (cws + 8 + 3) & ~(size_t)3;
    const size_t w4 = ((size_t)w + 3) & ~(size_t)3;
    const size_t ldb = ((size_t)(w - 1 + g.V - 1) + cws + w + g.V + 3) & ~(size_t)3;
    const size_t dist = 4 * w4 + 4 * c4 + c4 + (size_t)g.RCH * BMW + (size_t)g.RCH * ldb + RPAD;
    const size_t sel = cwt4 + (size_t)(CAP + 1) * g.NT + (size_t)(g.NT / 64) * COOP_FLOATS;
    return dist > sel ? dist : sel;
}

// The sub-tile's diagonals (SBW + 2w - 2, plus up to V-1 below diagonal 0
// that align the lower triangle to the blocks) must fit the threads' blocks of V,
// and a row's blocks the lanes given to it (two blocks per lane at most).
bool geometry_ok(int w, const Geo &g) {
    const int cws = g.SBW + w - 1;
    const int nbl = (cws + G - 1) / G;
    const int rpw = g.RCH > g.NT / 64 ? g.RCH / (g.NT / 64) : 1;
    const int lpr = 64 / rpw;
    return w <= kMaxW && g.V * g.NT >= cws + w - 1 + g.V - 1 && cws + g.V + 2 <= kStageIters * g.NT && g.SBW <= lpr * G && nbl <= 2 * lpr && nbl <= BMW &&
           4 * lds_floats(w, g) <= (g.NT == 256 ? kLdsTwo : kLdsOne);
}

// Two 256-thread workgroups per CU where their LDS fits (so one can select
// while the other computes), else one of 512 threads.
Geo geo_heuristic(int w) {
    Geo g;
    g.NT = 256;
    g.nA = 256;
    g.SBW = 32 * G;
    g.JT = g.nA * G;
    g.RCH = 8;
    g.V = g.SBW + 2 * w - 2 + 4 <= 5 * 256 ? 5 : 6;
    if (geometry_ok(w, g)) return g;
    g.NT = 512;
    if (w <= 513) {  // all threads select: fastest at w = 257 and 513 (of every candidate)
        g.nA = 512;
        g.SBW = 64 * G;
    } else {
        g.nA = 256;
        g.SBW = 32 * G;
    }
    g.JT = g.nA * G;
    g.V = g.SBW + 2 * w - 2 + 4 <= 5 * 512 ? 5 : 6;
    // rows per chunk: 8, or 4 where the row buffer does not fit or the
    // register blocks are 6 wide
    g.RCH = 8;
    if (g.V == 6 || 4 * lds_floats(w, g) > kLdsOne) g.RCH = 4;
    return g;
}

// A geometry as one number: threads/256 << 24 | V << 16 | RCH << 8 |
// nA/256 << 4 | SBW/(32 G).
int32_t geo_code(const Geo &g) {
    return ((g.NT / 256) << 24) | (g.V << 16) | (g.RCH << 8) | ((g.nA / 256) << 4) | (g.SBW / (32 * G));
}
Geo geo_decode(int32_t c) {
    Geo g;
    g.NT = ((c >> 24) & 0xF) * 256;
    g.V = (c >> 16) & 0xFF;
    g.RCH = (c >> 8) & 0xFF;
    g.nA = ((c >> 4) & 0xF) * 256;
    g.SBW = (c & 0xF) * 32 * G;
    g.JT = g.nA * G;
    return g;
}

// Every geometry the instantiated kernels can run for w: (threads, diagonals
// per thread, rows per chunk) of a kernel, 256 or 512
// selection threads (at most the workgroup's), sub-tiles of 992 or 1984
// windows, within the limits of geometry_ok.
int geo_candidates(int w, int32_t *codes, int max) {
    static const int kern[][3] = {{256, 5, 8}, {256, 6, 8}, {512, 5, 8}, {512, 5, 4}, {512, 6, 4}};
    int n = 0;
    for (const auto &k : kern)
        for (int na = 256; na <= k[0]; na += 256)
            for (int sb = 1; sb <= 2; ++sb) {
                Geo g;
                g.NT = k[0];
                g.V = k[1];
                g.RCH = k[2];
                g.nA = na;
                g.SBW = sb * 32 * G;
                g.JT = na * G;
                if (!geometry_ok(w, g)) continue;
                if (n < max) codes[n] = geo_code(g);
                ++n;
            }
    return n;
}

// Geometries chosen by the autotuner, per w (0: the heuristic).
std::atomic<int32_t> g_geo_code[kMaxW + 1];

Geo geo_for(int w) {
    const int32_t c = w >= 1 && w <= kMaxW ? g_geo_code[w].load(std::memory_order_relaxed) : 0;
    return c ? geo_decode(c) : geo_heuristic(w);
}

}  // namespace

int32_t profile_geometry(int32_t w) { return geo_code(geo_for(w)); }

int32_t profile_geometry_candidates(int32_t w, int32_t *codes, int32_t max) {
    return w >= 1 && w <= kMaxW ? geo_candidates(w, codes, max) : 0;
}

bool profile_set_geometry(int32_t w, int32_t code) {
    if (w < 1 || w > kMaxW) return false;
    if (code != 0) {
        int32_t c[64];
        const int n = geo_candidates(w, c, 64);
        bool ok = false;
        for (int i = 0; i < n && i < 64; ++i) ok |= c[i] == code;
        if (!ok) return false;
    }
    g_geo_code[w].store(code, std::memory_order_relaxed);
    return true;
}

int32_t profile_tile_windows(int32_t w) { return geo_for(w).JT; }

int32_t profile_slots(int32_t w) { return kCUs * (512 / geo_for(w).NT); }

int32_t profile_shape(int32_t w) { return geo_code(geo_for(w)); }

int32_t profile_grid(int64_t tiles, int32_t w) {
    const int64_t slots = profile_slots(w);
    return (int32_t)(tiles < slots ? (tiles > 0 ? tiles : 1) : slots);
}

// scratch floats of one workgroup: the row minima of a tile, then the tile's
// column minima
static size_t slot_floats_geo(int32_t w, const Geo &g) {
    const size_t JT = (size_t)g.JT;
    return (size_t)w * JT + ((JT + w - 1 + 3) & ~(size_t)3);
}
static size_t slot_floats_for(int32_t w) { return slot_floats_geo(w, geo_for(w)); }

// The largest profile scratch any candidate geometry needs for nq queries of
// Nm windows at w (workspaces are sized with it, so that a geometry chosen
// later still fits).
size_t profile_scratch_bound(int64_t Nm, int64_t nq, int32_t w) {
    int32_t c[64];
    const int n = std::min(geo_candidates(w, c, 64), 64);
    size_t best = 0;
    auto one = [&](const Geo &g) {
        const int64_t tiles = ((Nm + g.JT - 1) / g.JT) * nq;
        const int64_t slots = kCUs * (512 / g.NT);
        const int64_t grid = std::max<int64_t>(1, std::min(tiles, slots));
        best = std::max(best, (size_t)grid * slot_floats_geo(w, g));
    };
    for (int i = 0; i < n; ++i) one(geo_decode(c[i]));
    one(geo_heuristic(w));
    return best;
}

size_t profile_scratch_floats(int32_t grid, int32_t w) { return (size_t)grid * slot_floats_for(w); }

size_t profile_lds_bytes(int32_t w) { return 4 * lds_floats(w, geo_for(w)); }

int64_t profile_tiles(const ProfileJob &j) {
    const int JT = geo_for(j.w).JT;
    return ((j.Nm + JT - 1) / JT) * (int64_t)j.nq;
}

static_assert(sizeof(ProfileArgs) <= 4000, "kernel arguments must fit the 4 KB limit");

static const void *kernel_for(const Geo &g) {
    if (g.NT == 256) return g.V == 5 ? (const void *)k_profile<256, 5, 8> : (const void *)k_profile<256, 6, 8>;
    if (g.V == 5) return g.RCH == 8 ? (const void *)k_profile<512, 5, 8> : (const void *)k_profile<512, 5, 4>;
    return (const void *)k_profile<512, 6, 4>;
}

hipError_t profile_prepare(int32_t wmax) {
    const Geo g = geo_for(wmax);
    const size_t lds = 4 * lds_floats(wmax, g);
    return hipFuncSetAttribute(kernel_for(g), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

hipError_t launch_profile_batch(const ProfileJob *jobs, int n, int32_t grid, uint32_t *counter,
                                hipStream_t st) {
    if (n < 1 || n > kMaxJobs || grid < 1) return hipErrorInvalidValue;
    int wmax = 0;
    for (int i = 0; i < n; ++i) wmax = jobs[i].w > wmax ? jobs[i].w : wmax;
    const Geo g = geo_for(wmax);
    ProfileArgs a;
    a.g = g;
    a.B.njobs = n;
    a.B.slot_floats = slot_floats_for(wmax);
    a.B.counter = counter;
    int64_t acc = 0;
    for (int i = 0; i < n; ++i) {
        // all jobs of a batch share the geometry of the widest one
        a.B.J[i] = jobs[i];
        acc += ((jobs[i].Nm + g.JT - 1) / g.JT) * (int64_t)jobs[i].nq;
        a.B.tile_end[i] = acc;
    }
    const size_t lds = 4 * lds_floats(wmax, g);
    if (!geometry_ok(wmax, g)) return hipErrorInvalidValue;
    void *args[] = {&a};
    return hipLaunchKernel(kernel_for(g), dim3(grid), dim3(g.NT), args, lds, st);
}

hipError_t launch_profile(const ProfileJob &job, hipStream_t st) {
    hipError_t e = profile_prepare(job.w);
    if (e != hipSuccess) return e;
    return launch_profile_batch(&job, 1, job.grid, nullptr, st);
}

}  // namespace pst

#ifdef PST_PROBE
// Sums of the probe counters since the last reset: 0 windows, 1 run starts,
// 2 windows solved by their own bracket pass, 3 cooperative selects, 4-7
// misses with the k-th value below the bracket, above it, with an
// overflowing list, at a run's first window; 8 overflows of a one-key
// bracket, 9 the sum of the list lengths, 10 overflows that held the k-th
// value, 11 windows with a second-pass bracket, 12 windows a second pass
// solved; wave
// cycles of 16 the distance phase, 17 FP64 anchors, 18 the FP32 recurrence,
// 19 column minima, 20 sliding row minima, 21 the selection phase, 22 run
// starts, 23 first bracket passes, 24 sorts and second passes, 25 cooperative
// selects.
extern "C" int pst_probe_read(unsigned long long *out, int reset) {
    static unsigned long long buf[32 * 64];
    if (hipMemcpyFromSymbol(buf, HIP_SYMBOL(g_probe), sizeof(buf)) != hipSuccess) return -3;
    for (int i = 0; i < 32; ++i) {
        out[i] = 0;
        for (int j = 0; j < 64; ++j) out[i] += buf[i * 64 + j];
    }
    if (reset) {
        static const unsigned long long zero[32 * 64] = {};
        if (hipMemcpyToSymbol(HIP_SYMBOL(g_probe), zero, sizeof(zero)) != hipSuccess) return -3;
    }
    return 0;
}
#endif

