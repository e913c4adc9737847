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
// therefore works on y = 1 - rho (d^2 = 2 l y) and forms one distance per
// window, from the selected y.
//
// Work unit: a tile of (query, JT consecutive windows), JT = 31 * (number of
// selection threads).  The tile is computed in sub-tiles of SBW windows; a
// sub-tile needs the w x (SBW + w - 1) block of the matrix:
//   1. FP64 anchors: the centred covariance at the first cell of each diagonal
//      of the block, by a direct dot product (register-blocked along the row).
//   2. Rows in chunks of V: each thread owns V adjacent diagonals and advances
//      them one row at a time with the FP32 centred-covariance recurrence
//          cov(r+1, c+1) = cov(r, c) + df[r]*dg[c] + df[c]*dg[r];
//      the statistics of its V columns sit in a register window that slides by
//      one column per row.  The chunk's y values go to LDS.
//   3. Column minima of y accumulate in LDS for the whole tile (eq. 10).
//   4. Sliding row minima of width w (eq. 11), per (row, block of 31 windows):
//      suffix minima of the block and running minima of the window tails in
//      registers, whole blocks in between from per-block minima in LDS.  They
//      go to a per-workgroup scratch slot, block-interleaved so that both the
//      writes here and the reads below are coalesced.
//   5. Selection (eqs. 12-13): thread a takes the 31 windows of block a, in
//      order.  A run starts with an MSD radix select on the bits of y that
//      brackets the ranks k-8 .. k+8 and sorts the values inside; each next
//      window makes one pass that counts the values below that bracket and
//      collects the ones inside it (adjacent windows share all but a few of
//      their 2w values, so the k-th value rarely leaves the bracket), and
//      takes the next bracket from the sorted list.  Windows whose bracket
//      misses (and the first window of each run) are solved by the 64 lanes of
//      the wave together, one window at a time, with the radix select, so a
//      rare miss costs the wave a short cooperative step instead of stalling
//      every lane.  The result is exact either way.
//
// Arithmetic of a cell depends only on the query's data, the column and the
// window offset inside the tile, never on the query's position, so identical
// segments get bit-identical profiles.
#include "pst_internal.h"

#include <math.h>

namespace pst {
namespace {

constexpr int NT = kProfileThreads;
constexpr int G = 31;      // windows per block (odd: conflict-free LDS strides)
constexpr int CAP = 28;    // sorted candidate list capacity
constexpr int NB = 16;     // radix buckets per level
constexpr int BAND = 8;    // bracket half-width in ranks

struct Geo {
    int JT;     // windows per tile
    int nA;     // selection threads = blocks per tile = JT / G
    int SBW;    // windows per sub-tile (multiple of G)
    int V;      // diagonals per thread
};

struct ProfileArgs {
    ProfileBatch B;
    Geo g;
};

__device__ __forceinline__ uint32_t ykey(float y) { return __float_as_uint(fmaxf(y, 0.0f)); }

// In-place insertion sort of the n values L[0], L[NT], ... (per-thread list).
__device__ __forceinline__ void sort_list(float *L, int n) {
    for (int x = 1; x < n; ++x) {
        const float key = L[x * NT];
        int j = x - 1;
        while (j >= 0 && L[j * NT] > key) {
            L[(j + 1) * NT] = L[j * NT];
            --j;
        }
        L[(j + 1) * NT] = key;
    }
}

// Values of one window: A(i) for i < w (row minima) and B(c) for c < w
// (column minima).  each() visits every value exactly once.
struct Window {
    const float *rw;   // scratch slot
    int aoff, astr;    // A(i) = rw[aoff + i * astr]
    const float *bv;   // B(c) = bv[c]
    int w;
    template <typename F>
    __device__ __forceinline__ void each(F f) const {
        int i = 0;
        for (; i + 16 <= w; i += 16) {
            float y[16];
#pragma unroll
            for (int e = 0; e < 16; ++e) y[e] = rw[aoff + (i + e) * astr];
#pragma unroll
            for (int e = 0; e < 16; ++e) f(y[e]);
        }
        for (; i < w; ++i) f(rw[aoff + i * astr]);
        int c = 0;
        for (; c + 16 <= w; c += 16) {
            float y[16];
#pragma unroll
            for (int e = 0; e < 16; ++e) y[e] = bv[c + e];
#pragma unroll
            for (int e = 0; e < 16; ++e) f(y[e]);
        }
        for (; c < w; ++c) f(bv[c]);
    }
};

// Orders LDS accesses of the lanes of one wave (they execute in lockstep).
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Per-wave LDS scratch of the cooperative select.
struct Coop {
    unsigned *hist;   // NB counters
    unsigned *cnt;    // 1 counter
    float *list;      // CAP values
    float *sorted;    // CAP values
};
constexpr int COOP_FLOATS = NB + 4 + 2 * CAP;

// Exact radix select, by the 64 lanes of a wave together, of the key range
// holding ranks r1 .. r2 (1-based) of one window's 2w values: A(i) =
// rw[aoff + i*astr] for i < w and B(c) = bv[c] for c < w.  Every lane gets
// *below (values under the range) and the count of values in it; those values
// are left sorted in C.sorted.  If the range cannot be narrowed to CAP values
// the ranks shrink to k .. k.  Must be called by all lanes of the wave.
__device__ __forceinline__ int coop_band(const float *rw, int aoff, int astr, const float *bv, int w, int k, int r1,
                         int r2, const Coop &C, int lane, int *below) {
    uint32_t lo = 0u, hi = 0x7F800000u;
    int base = 0, shift = -1;
    for (int level = 0; level < 16; ++level) {
        if (lane < NB) C.hist[lane] = 0u;
        wave_sync();
        auto add = [&](float y) {
            const uint32_t key = ykey(y);
            if (key >= lo && key < hi) {
                int b;
                if (shift < 0) b = min(max(((int)(key >> 23) - 96) >> 1, 0), NB - 1);
                else b = (int)((key - lo) >> shift);
                atomicAdd(&C.hist[b], 1u);
            }
        };
        for (int i = lane; i < w; i += 64) add(rw[aoff + i * astr]);
        for (int c = lane; c < w; c += 64) add(bv[c]);
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
        uint32_t nlo, nhi;
        if (shift < 0) {
            nlo = b1 == 0 ? 0u : (uint32_t)(2 * b1 + 96) << 23;
            nhi = b2 == NB - 1 ? 0x7F800000u : (uint32_t)(2 * b2 + 98) << 23;
        } else {
            nlo = lo + ((uint32_t)b1 << shift);
            const uint64_t e = (uint64_t)lo + ((uint64_t)(b2 + 1) << shift);
            nhi = (uint32_t)(e < (uint64_t)hi ? e : (uint64_t)hi);
        }
        const bool stuck = (nlo == lo && nhi == hi);
        lo = nlo;
        hi = nhi;
        base = below1;
        wave_sync();  // every lane has read the histogram
        if (hi - lo == 1u) {  // one key value holds ranks r1 .. r2
            if (lane == 0) C.sorted[0] = __uint_as_float(lo);
            wave_sync();
            *below = base;
            return 1;
        }
        if (cnt <= CAP) {
            if (lane == 0) *C.cnt = 0u;
            wave_sync();
            auto col = [&](float y) {
                const uint32_t key = ykey(y);
                if (key >= lo && key < hi) C.list[atomicAdd(C.cnt, 1u)] = __uint_as_float(key);
            };
            for (int i = lane; i < w; i += 64) col(rw[aoff + i * astr]);
            for (int c = lane; c < w; c += 64) col(bv[c]);
            wave_sync();
            if (lane < cnt) {  // rank of each value, ties by position
                const float y = C.list[lane];
                int r = 0;
                for (int x = 0; x < cnt; ++x) {
                    const float yx = C.list[x];
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
        const uint32_t span = hi - lo;
        const int lg = 32 - __clz((int)(span - 1u));
        shift = max(0, lg - 4);
    }
    *below = base;  // not reached for finite keys
    if (lane == 0) C.sorted[0] = __uint_as_float(lo);
    wave_sync();
    return 1;
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

template <int V>
__global__ void __launch_bounds__(NT) k_profile(ProfileArgs A) {
    extern __shared__ __align__(16) float sm[];
    __shared__ uint32_t next_tile;
    const Geo g = A.g;
    const int JT = g.JT, nA = g.nA, SBW = g.SBW;
    const int t = threadIdx.x;
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
        const int w4 = (w + 3) & ~3;
        const int CWT = JT + w - 1;          // columns of a tile
        const int CWS = SBW + w - 1;         // columns of a sub-tile
        const float two_l = (float)(2 * l);

        // LDS: column minima of the tile and row statistics, then a region
        // shared by the sub-tile distance phase and the selection phase.
        float *colY = sm;
        float *r_inv = colY + ((CWT + 3) & ~3);
        float *r_df = r_inv + w4;
        float *r_dg = r_df + w4;
        float *r_h = r_dg + w4;
        float *Ureg = r_h + w4;
        float *c_inv = Ureg;
        float *c_df = c_inv + CWS;
        float *c_dg = c_df + CWS;
        float *c_h = c_dg + CWS;
        float *buf = c_h + CWS;      // V rows x CWS
        float *BM = buf + V * CWS;   // V rows x blocks
        float *lst = Ureg;                  // selection: CAP x NT per-thread lists
        float *coop = lst + CAP * NT;       // then per-wave scratch

        float *rw = J.rw + (size_t)blockIdx.x * A.B.slot_floats;
        float tmax = 0.0f;

        const int s = (int)(tile / ntile);
        const int64_t J0 = (tile % ntile) * JT;
        const int JTe = (int)min<int64_t>(JT, J.Nm - J0);
        const int CW = JTe + w - 1;
        const int64_t rb = (int64_t)s * J.row_stride;

        __syncthreads();  // the previous tile is done with LDS and the scratch slot
        for (int u = t; u < CW; u += NT) colY[u] = INFINITY;
        for (int i = t; i < w; i += NT) {
            const int64_t r = rb + i;
            r_inv[i] = J.row.inv[r];
            r_df[i] = J.row.df[r];
            r_dg[i] = J.row.dg[r];
            r_h[i] = J.row.h[r];
        }

        for (int Js = 0; Js < JTe; Js += SBW) {
            const int JSe = min(SBW, JTe - Js);   // windows of this sub-tile
            const int CS = JSe + w - 1;           // its columns
            const int nbl = (CS + G - 1) / G;
            const bool last = Js + SBW >= JTe;
            const int own = last ? CS : SBW;      // columns whose minima it owns
            const int64_t C0 = J0 + Js;           // first column (series index)
            __syncthreads();  // previous sub-tile done with the shared region
            for (int u = t; u < CS; u += NT) {
                const int64_t c = C0 + u;
                c_inv[u] = J.col.inv[c];
                c_df[u] = J.col.df[c];
                c_dg[u] = J.col.dg[c];
                c_h[u] = J.col.h[c];
            }

            // 1. FP64 anchors of this thread's V diagonals d0 .. d0+V-1;
            //    diagonal d holds the cells (i, u = d - (w-1) + i), 0 <= u < CS.
            const int d0 = t * V;
            const int ub0 = d0 - (w - 1);
            const bool full = (ub0 >= 0) && (d0 + V - 1 <= CS - 1);
            float cov[V];
            if (full) {
                const double *xr = J.row.xc + rb;
                const double *xcp = J.col.xc + C0 + ub0;
                double acc[V], xs[V];
#pragma unroll
                for (int v = 0; v < V; ++v) acc[v] = 0.0;
#pragma unroll
                for (int v = 0; v < V - 1; ++v) xs[v] = xcp[v];
                int tt = 0;
                for (; tt + V <= l; tt += V) {
#pragma unroll
                    for (int kq = 0; kq < V; ++kq) {
                        xs[(kq + V - 1) % V] = xcp[tt + kq + V - 1];
                        const double a = xr[tt + kq];
#pragma unroll
                        for (int v = 0; v < V; ++v) acc[v] = fma(a, xs[(kq + v) % V], acc[v]);
                    }
                }
                for (; tt < l; ++tt) {
                    const double a = xr[tt];
#pragma unroll
                    for (int v = 0; v < V; ++v) acc[v] = fma(a, xcp[tt + v], acc[v]);
                }
                const double mr = (double)l * J.row.mu[rb];
#pragma unroll
                for (int v = 0; v < V; ++v) cov[v] = (float)(acc[v] - mr * J.col.mu[C0 + ub0 + v]);
            } else {
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    const int d = d0 + v;
                    cov[v] = 0.0f;
                    if (d < CS + w - 1) {
                        const int i0 = max(0, w - 1 - d);
                        const int u0 = d - (w - 1) + i0;
                        const double *xr = J.row.xc + rb + i0;
                        const double *xcp = J.col.xc + C0 + u0;
                        double acc = 0.0;
                        for (int tt = 0; tt < l; ++tt) acc = fma(xr[tt], xcp[tt], acc);
                        cov[v] = (float)(acc - (double)l * J.row.mu[rb + i0] * J.col.mu[C0 + u0]);
                    }
                }
            }
            __syncthreads();

            // register window of column statistics: slot (v + k) % V holds the
            // column of diagonal v at row phase k
            float wi[V], wf[V], wg[V], wh[V];
#pragma unroll
            for (int v = 0; v < V; ++v) {
                const int u = min(max(ub0 + v, 0), CS - 1);
                wi[v] = c_inv[u];
                wf[v] = c_df[u];
                wg[v] = c_dg[u];
                wh[v] = c_h[u];
            }

            for (int R0 = 0; R0 < w; R0 += V) {
                const int nr = min(V, w - R0);
                // 2. rows R0 .. R0+nr-1 of y = 1 - rho
#pragma unroll
                for (int k = 0; k < V; ++k) {
                    const int i = R0 + k;
                    if (i < w) {
                        if (i > 0) {
                            const int sl = (k + V - 1) % V;
                            const int u = min(max(ub0 + V - 1 + i, 0), CS - 1);
                            wi[sl] = c_inv[u];
                            wf[sl] = c_df[u];
                            wg[sl] = c_dg[u];
                            wh[sl] = c_h[u];
                        }
                        if (J.anchor_every > 0 && i > 0 && i % J.anchor_every == 0) {
                            // optional FP64 re-anchor: the FP32 recurrence never
                            // runs more than anchor_every steps
#pragma unroll
                            for (int v = 0; v < V; ++v) {
                                const int u = ub0 + v + i;
                                if (u >= 0 && u < CS) cov[v] = anchor_at(J, rb, i, C0, u);
                            }
                        }
                        const float ri = r_inv[i], rf = r_df[i], rg = r_dg[i], rh1 = 1.0f - r_h[i];
                        float *brow = buf + k * CS;
                        if (full) {
#pragma unroll
                            for (int v = 0; v < V; ++v) {
                                const int sl = (v + k) % V;
                                brow[ub0 + v + i] = fmaf(-cov[v] * ri, wi[sl], rh1 - wh[sl]);
                                cov[v] = fmaf(rf, wg[sl], fmaf(wf[sl], rg, cov[v]));
                            }
                        } else {
#pragma unroll
                            for (int v = 0; v < V; ++v) {
                                const int sl = (v + k) % V;
                                const int u = ub0 + v + i;
                                if (u >= 0) {
                                    if (u < CS) brow[u] = fmaf(-cov[v] * ri, wi[sl], rh1 - wh[sl]);
                                    cov[v] = fmaf(rf, wg[sl], fmaf(wf[sl], rg, cov[v]));
                                }
                            }
                        }
                    }
                }
                __syncthreads();
                // 3. column minima of y (eq. 10) for the columns this sub-tile owns
                for (int u = t; u < own; u += NT) {
                    float mn = colY[Js + u];
                    for (int rr = 0; rr < nr; ++rr) mn = fminf(mn, buf[rr * CS + u]);
                    colY[Js + u] = mn;
                }
                // 4. sliding row minima of width w (eq. 11)
                const int rr = t / nbl;
                const int al = t - rr * nbl;   // block inside the sub-tile
                const bool act = rr < nr;
                float S[G];
                if (act) {
                    const float *src = buf + rr * CS + al * G;
                    const int lim = CS - al * G;
#pragma unroll
                    for (int j = 0; j < G; ++j) S[j] = j < lim ? src[j] : INFINITY;
#pragma unroll
                    for (int j = G - 2; j >= 0; --j) S[j] = fminf(S[j], S[j + 1]);
                    BM[rr * nbl + al] = S[0];
                }
                __syncthreads();
                if (act && al * G < JSe) {
                    const float *row = buf + rr * CS;
                    const int a = Js / G + al;                 // block inside the tile
                    const int obase = (R0 + rr) * G * nA + a;  // + p * nA
                    const int vend = min(G, JSe - al * G);
                    if (w <= G) {
                        for (int p = 0; p < vend; ++p) {
                            const int v = al * G + p;
                            float mn = INFINITY;
                            for (int c = 0; c < w; ++c) mn = fminf(mn, row[v + c]);
                            rw[obase + p * nA] = mn;
                        }
                    } else {
                        const int q = (w - 1) / G;
                        const int rp = (w - 1) - q * G;
                        float base = INFINITY;
                        for (int b = al + 1; b < al + q; ++b) base = fminf(base, BM[rr * nbl + b]);
                        const int pb = (al + q) * G;
                        for (int x = 0; x <= rp; ++x) base = fminf(base, row[pb + x]);
                        // tail: columns al*G + w - 1 + p for p = 1 .. G-1
                        const int tb = al * G + w - 1;
                        float pr = base;
#pragma unroll
                        for (int p = 0; p < G; ++p) {
                            if (p > 0) pr = fminf(pr, row[min(tb + p, CS - 1)]);
                            if (p < vend) rw[obase + p * nA] = fminf(S[p], pr);
                        }
                    }
                }
                __syncthreads();
            }
        }

        // 5. selection (eqs. 12-13): k-th smallest y of the w row minima and the
        //    w column minima of each window; thread a takes block a in order.
        //    Windows whose bracket misses are solved by the whole wave together.
        if (t < nA) {
            float *L = lst + t;
            const int lane = t & 63;
            float *cs = coop + (t >> 6) * COOP_FLOATS;
            const Coop C{(unsigned *)cs, (unsigned *)(cs + NB), cs + NB + 4, cs + NB + 4 + CAP};
            const int r1 = max(1, keff - BAND), r2 = min(2 * w, keff + BAND);
            bool have = false;
            float blo = 0.0f, bhi = 0.0f, ystar = 0.0f;
            const int astr = G * nA;
            for (int p = 0; p < G; ++p) {
                const int v = t * G + p;
                const bool valid = v < JTe;
                bool ok = false;
                if (valid && have) {
                    Window W{rw, p * nA + t, astr, colY + v, w};
                    int below = 0, nl = 0;
                    const float lo_ = blo, hi_ = bhi;
                    W.each([&](float y) {
                        below += y < lo_;
                        if (y >= lo_ && y <= hi_) {
                            if (nl < CAP) L[nl * NT] = y;
                            ++nl;
                        }
                    });
                    const int kk = keff - below;
                    if (kk >= 1 && kk <= nl && nl <= CAP) {
                        sort_list(L, nl);
                        ystar = L[(kk - 1) * NT];
                        // next bracket: ranks k-BAND .. k+BAND of this window, or
                        // extrapolated from the list's spacing where it ends early
                        const int q1 = r1 - below, q2 = r2 - below;
                        const float l0 = L[0], l1 = L[(nl - 1) * NT];
                        const float sp = (l1 - l0) / (float)max(nl - 1, 1);
                        blo = q1 >= 1 ? L[(q1 - 1) * NT] : l0 - 1.5f * (float)(1 - q1) * sp;
                        bhi = q2 <= nl ? L[(q2 - 1) * NT] : l1 + 1.5f * (float)(q2 - nl) * sp;
                        ok = true;
                    }
                }
                uint64_t need = __ballot(valid && !ok);
                while (need) {
                    const int ln = __ffsll((unsigned long long)need) - 1;
                    need &= need - 1;
                    const int tf = (t & ~63) + ln;
                    int below = 0;
                    const int nc = coop_band(rw, p * nA + tf, astr, colY + tf * G + p, w, keff, r1, r2,
                                             C, lane, &below);
                    if (lane == ln) {
                        const int kk = keff - below;
                        ystar = C.sorted[min(max(kk, 1), nc) - 1];
                        blo = C.sorted[min(max(r1 - below, 1), nc) - 1];
                        bhi = C.sorted[min(max(r2 - below, 1), nc) - 1];
                        have = true;
                    }
                    wave_sync();
                }
                if (valid) {
                    const float dist = sqrtf(two_l * fmaxf(ystar, 0.0f));
                    J.D[(int64_t)s * J.ld + J0 + v] = dist;
                    tmax = fmaxf(tmax, dist);
                }
            }
        }

        // max of D over this tile (the denominator of eq. 18): one atomic per wave
        if (J.dmax_bits) {
            float mx = tmax;
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o));
            if ((t & 63) == 0) atomicMax(J.dmax_bits, __float_as_uint(mx));
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

Geo geo_for(int w) {
    Geo g;
    if (w <= 257) {
        g.nA = 512;
        g.SBW = 64 * G;
    } else if (w <= 513) {
        g.nA = 256;
        g.SBW = 64 * G;
    } else {
        g.nA = 256;
        g.SBW = 32 * G;
    }
    g.JT = g.nA * G;
    const int ndiag = g.SBW + 2 * w - 2;
    g.V = ndiag <= 5 * NT ? 5 : 6;
    return g;
}

size_t lds_floats(int w, const Geo &g) {
    const size_t cwt = (((size_t)g.JT + w - 1) + 3) & ~(size_t)3;
    const size_t cws = (size_t)g.SBW + w - 1;
    const size_t nbl = (cws + G - 1) / G;
    const size_t w4 = ((size_t)w + 3) & ~(size_t)3;
    const size_t dist = 4 * cws + (size_t)g.V * cws + (size_t)g.V * nbl;
    const size_t sel = (size_t)CAP * NT + (size_t)(NT / 64) * COOP_FLOATS;
    return cwt + 4 * w4 + (dist > sel ? dist : sel);
}

}  // namespace

int32_t profile_tile_windows(int32_t w) { return geo_for(w).JT; }

int32_t profile_grid(int64_t tiles) {
    const int64_t slots = 256;  // one workgroup per compute unit
    return (int32_t)(tiles < slots ? (tiles > 0 ? tiles : 1) : slots);
}

size_t profile_scratch_floats(int32_t grid, int32_t w) {
    return (size_t)grid * w * profile_tile_windows(w);
}

size_t profile_lds_bytes(int32_t w) { return 4 * lds_floats(w, geo_for(w)); }

int64_t profile_tiles(const ProfileJob &j) {
    const int JT = geo_for(j.w).JT;
    return ((j.Nm + JT - 1) / JT) * (int64_t)j.nq;
}

static_assert(sizeof(ProfileArgs) <= 4000, "kernel arguments must fit the 4 KB limit");

hipError_t profile_prepare(int32_t wmax) {
    const Geo g = geo_for(wmax);
    const size_t lds = 4 * lds_floats(wmax, g);
    const void *fn = g.V == 5 ? (const void *)k_profile<5> : (const void *)k_profile<6>;
    return hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
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
    a.B.slot_floats = (size_t)wmax * g.JT;
    a.B.counter = counter;
    int64_t acc = 0;
    for (int i = 0; i < n; ++i) {
        // all jobs of a batch share the geometry of the widest one
        a.B.J[i] = jobs[i];
        acc += ((jobs[i].Nm + g.JT - 1) / g.JT) * (int64_t)jobs[i].nq;
        a.B.tile_end[i] = acc;
    }
    const size_t lds = 4 * lds_floats(wmax, g);
    const int cws = g.SBW + wmax - 1;
    const int nbl = (cws + G - 1) / G;
    // every (row, block) item of a row chunk maps to one thread; every
    // diagonal of a sub-tile to one thread's register block
    if (wmax > kMaxW || g.V * nbl > NT || g.V * NT < cws + wmax - 1 || lds > 158 * 1024)
        return hipErrorInvalidValue;
    if (g.V == 5) hipLaunchKernelGGL(k_profile<5>, dim3(grid), dim3(NT), lds, st, a);
    else hipLaunchKernelGGL(k_profile<6>, dim3(grid), dim3(NT), lds, st, a);
    return hipGetLastError();
}

hipError_t launch_profile(const ProfileJob &job, hipStream_t st) {
    hipError_t e = profile_prepare(job.w);
    if (e != hipSuccess) return e;
    return launch_profile_batch(&job, 1, job.grid, nullptr, st);
}

}  // namespace pst
