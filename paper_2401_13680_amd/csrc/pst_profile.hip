// The MPdist-profile kernel: eqs. 9-13 of section 4.1 for every (query, window).
//
// For query s (a segment S_s of T, eq. 4, or an external query Q) the kernel
// evaluates the distance matrix ED_matr (eq. 9) between the query's w = m-l+1
// length-l subsequences (rows) and the series' length-l subsequences
// (columns), its column minima allP_BA (eq. 10) and its row minima over a
// sliding window of w columns allP_AB (eq. 11), and for every length-m window
// j the k-th smallest element of the concatenation P_ABBA (eqs. 12-13).
//
// Work is cut into tiles of (query, 1024 consecutive windows); a tile needs the
// w x (1024 + w - 1) block of the matrix, which it computes along diagonals:
//   - the centred covariance of row r and column c is anchored by an FP64 dot
//     product at the first cell of each diagonal inside the tile, and then
//     advanced in FP32 with the recurrence
//         cov(r+1, c+1) = cov(r, c) + df[r]*dg[c] + df[c]*dg[r]
//     (df, dg from the statistics pass);
//   - every later step is an order statistic and monotone in the Pearson
//     correlation rho = cov / (l sigma_r sigma_c), so minima of distances are
//     computed as maxima of rho, and a distance d = sqrt(2 l (1 - rho)) is
//     formed only for the selected value.
// Rows are produced in chunks staged in LDS; column maxima accumulate in LDS;
// row sliding maxima use a doubling (sparse-table) sweep in LDS and go to a
// per-workgroup scratch slot; the k-th selection is a per-window MSD radix
// select on order-preserving 32-bit keys of (1 - rho), with per-thread
// histograms in LDS.
//
// Arithmetic of a cell depends only on the query's data, the column and the
// tile's window offset, never on the query's position: identical segments get
// bit-identical profiles.
#include "pst_internal.h"

#include <math.h>

namespace pst {
namespace {

constexpr int NT = kThreads;
constexpr int JT = kTileWindows;

__device__ __forceinline__ uint32_t sel_key(float rho) {
    float y = 1.0f - rho;
    y = fminf(fmaxf(y, 0.0f), 2.0f);
    return __float_as_uint(y);
}

// Level-0 bucket: 2 buckets per binade of y = 1 - rho, y in [2^-31, 2];
// smaller values share bucket 0, [1.5, 2] is bucket 63.
__device__ __forceinline__ int bucket0(uint32_t key) {
    int b = (int)(key >> 22) - 192;
    return min(max(b, 0), kBuckets - 1);
}

struct ProfileArgs {
    ProfileJob J;
    int32_t rc;       // rows per LDS chunk
    int32_t cwmax;    // JT + w - 1
    float two_l;
};

__global__ void __launch_bounds__(NT) k_profile(ProfileArgs A) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const ProfileJob &J = A.J;
    const int w = J.w, l = J.l, RC = A.rc, CWM = A.cwmax;
    const int t = threadIdx.x;
    const int64_t ntile = (J.Nm + JT - 1) / JT;
    const int64_t total = ntile * (int64_t)J.nq;
    const int keff = min(J.k, 2 * w);

    float *c_inv = (float *)smem_raw;
    float *c_h = c_inv + CWM;
    float *c_df = c_h + CWM;
    float *c_dg = c_df + CWM;
    float *colmax = c_dg + CWM;
    float *r_inv = colmax + CWM;
    float *r_h = r_inv + w;
    float *r_df = r_h + w;
    float *r_dg = r_df + w;
    float *buf0 = r_dg + w;
    float *buf1 = buf0 + RC * CWM;
    unsigned *hist = (unsigned *)buf0;       // reused after the rows are done
    unsigned *list = hist + kBuckets * NT;

    float *rw = J.rw + (size_t)blockIdx.x * (size_t)w * JT;
    float tmax = 0.0f;

    for (int64_t tile = blockIdx.x; tile < total; tile += gridDim.x) {
        const int s = (int)(tile / ntile);
        const int64_t J0 = (tile % ntile) * JT;
        const int JTe = (int)min<int64_t>(JT, J.Nm - J0);
        const int CW = JTe + w - 1;
        const int ndiag = CW + w - 1;
        const int64_t rb = (int64_t)s * J.row_stride;

        __syncthreads();  // previous tile is done with LDS and its scratch slot
        for (int u = t; u < CW; u += NT) {
            const int64_t c = J0 + u;
            c_inv[u] = J.col.inv[c];
            c_h[u] = J.col.h[c];
            c_df[u] = J.col.df[c];
            c_dg[u] = J.col.dg[c];
            colmax[u] = -INFINITY;
        }
        for (int i = t; i < w; i += NT) {
            const int64_t r = rb + i;
            r_inv[i] = J.row.inv[r];
            r_h[i] = J.row.h[r];
            r_df[i] = J.row.df[r];
            r_dg[i] = J.row.dg[r];
        }

        // FP64 anchors: centred covariance at the first cell of each diagonal.
        float cov[kMaxDiagPerThread];
#pragma unroll
        for (int q = 0; q < kMaxDiagPerThread; ++q) {
            const int d = t + q * NT;
            cov[q] = 0.0f;
            if (d < ndiag) {
                const int i0 = max(0, w - 1 - d);
                const int u0 = d - (w - 1) + i0;
                const int64_t r = rb + i0;
                const int64_t c = J0 + u0;
                const double *xr = J.row.xc + r;
                const double *xcp = J.col.xc + c;
                double acc = 0.0;
                for (int tt = 0; tt < l; ++tt) acc = fma(xr[tt], xcp[tt], acc);
                acc -= (double)l * J.row.mu[r] * J.col.mu[c];
                cov[q] = (float)acc;
            }
        }
        __syncthreads();

        for (int R0 = 0; R0 < w; R0 += RC) {
            const int nr = min(RC, w - R0);
            // distance-matrix rows R0 .. R0+nr-1 as correlations
#pragma unroll
            for (int q = 0; q < kMaxDiagPerThread; ++q) {
                const int d = t + q * NT;
                if (d < ndiag) {
                    const int i0 = max(0, w - 1 - d);
                    const int iend = min(w, CW + w - 1 - d);
                    const int ilo = max(R0, i0), ihi = min(R0 + nr, iend);
                    float cv = cov[q];
                    for (int i = ilo; i < ihi; ++i) {
                        const int u = d - (w - 1) + i;
                        const float rho = fmaf(cv * r_inv[i], c_inv[u], r_h[i] + c_h[u]);
                        buf0[(i - R0) * CW + u] = rho;
                        cv = fmaf(r_df[i], c_dg[u], fmaf(c_df[u], r_dg[i], cv));
                    }
                    cov[q] = cv;
                }
            }
            __syncthreads();
            // eq. 10 (as a maximum of rho): column maxima over the rows so far
            for (int u = t; u < CW; u += NT) {
                float mx = colmax[u];
                for (int rr = 0; rr < nr; ++rr) mx = fmaxf(mx, buf0[rr * CW + u]);
                colmax[u] = mx;
            }
            // eq. 11 (as a maximum of rho): sliding maxima of width w by doubling
            float *src = buf0, *dst = buf1;
            int h = 1;
            while (2 * h <= w) {
                for (int e = t; e < nr * CW; e += NT) {
                    const int u = e % CW;
                    if (u + h < CW) dst[e] = fmaxf(src[e], src[e + h]);
                }
                __syncthreads();
                float *tmp = src;
                src = dst;
                dst = tmp;
                h *= 2;
            }
            const int off = w - h;
            for (int e = t; e < nr * JTe; e += NT) {
                const int rr = e / JTe, v = e % JTe;
                rw[(size_t)(R0 + rr) * JT + v] = fmaxf(src[rr * CW + v], src[rr * CW + v + off]);
            }
            __syncthreads();
        }

        // eqs. 12-13: k-th smallest distance = k-th largest rho of the 2w values
        unsigned *H = hist + t;
        unsigned *L = list + t;
        for (int v = t; v < JTe; v += NT) {
            const float *rwv = rw + v;
            const float *cmv = colmax + v;
            int kk = keff;
            uint32_t lo = 0u, hi = 0x40000001u, ans = 0u;
            int shift = -1;
            for (int level = 0; level < 8; ++level) {
                for (int b = 0; b < kBuckets; ++b) H[b * NT] = 0u;
                for (int i = 0; i < w; ++i) {
                    const uint32_t key = sel_key(rwv[(size_t)i * JT]);
                    if (key >= lo && key < hi) {
                        const int b = shift < 0 ? bucket0(key) : (int)((key - lo) >> shift);
                        H[b * NT] += 1u;
                    }
                }
                for (int c = 0; c < w; ++c) {
                    const uint32_t key = sel_key(cmv[c]);
                    if (key >= lo && key < hi) {
                        const int b = shift < 0 ? bucket0(key) : (int)((key - lo) >> shift);
                        H[b * NT] += 1u;
                    }
                }
                int acc = 0, bs = kBuckets - 1;
                unsigned cnt = 0u;
                for (int b = 0; b < kBuckets; ++b) {
                    const unsigned cb = H[b * NT];
                    if (acc + (int)cb >= kk) {
                        bs = b;
                        cnt = cb;
                        break;
                    }
                    acc += (int)cb;
                }
                kk -= acc;
                uint32_t nlo, nhi;
                if (shift < 0) {
                    nlo = bs == 0 ? 0u : (uint32_t)(bs + 192) << 22;
                    nhi = bs == kBuckets - 1 ? 0x40000001u : (uint32_t)(bs + 193) << 22;
                } else {
                    nlo = lo + ((uint32_t)bs << shift);
                    const uint64_t e = (uint64_t)nlo + (1ull << shift);
                    nhi = (uint32_t)(e < (uint64_t)hi ? e : (uint64_t)hi);
                }
                lo = nlo;
                hi = nhi;
                ans = lo;
                if (hi - lo == 1u) break;
                if ((int)cnt <= kCap) {
                    int nc = 0;
                    for (int i = 0; i < w; ++i) {
                        const uint32_t key = sel_key(rwv[(size_t)i * JT]);
                        if (key >= lo && key < hi) L[(nc++) * NT] = key;
                    }
                    for (int c = 0; c < w; ++c) {
                        const uint32_t key = sel_key(cmv[c]);
                        if (key >= lo && key < hi) L[(nc++) * NT] = key;
                    }
                    for (int a = 0; a < nc; ++a) {
                        const uint32_t ka = L[a * NT];
                        int less = 0, leq = 0;
                        for (int b = 0; b < nc; ++b) {
                            const uint32_t kb = L[b * NT];
                            less += kb < ka;
                            leq += kb <= ka;
                        }
                        if (less < kk && kk <= leq) {
                            ans = ka;
                            break;
                        }
                    }
                    break;
                }
                const uint32_t span = hi - lo;
                const int lg = 32 - __clz((int)(span - 1u));
                shift = max(0, lg - 6);
            }
            const float y = __uint_as_float(ans);
            const float dist = sqrtf(A.two_l * y);
            J.D[(int64_t)s * J.ld + J0 + v] = dist;
            tmax = fmaxf(tmax, dist);
        }
    }

    if (J.dmax_bits) {
        __shared__ float red[NT];
        __syncthreads();
        red[t] = tmax;
        __syncthreads();
        for (int o = NT / 2; o > 0; o >>= 1) {
            if (t < o) red[t] = fmaxf(red[t], red[t + o]);
            __syncthreads();
        }
        if (t == 0) atomicMax(J.dmax_bits, __float_as_uint(red[0]));
    }
}

size_t lds_bytes(int w, int rc) {
    const size_t cwm = (size_t)JT + w - 1;
    const size_t fixed = 4 * (5 * cwm + 4 * (size_t)w);
    const size_t rows = 2 * (size_t)rc * cwm * 4;
    const size_t sel = (size_t)(kBuckets + kCap) * NT * 4;
    return fixed + (rows > sel ? rows : sel);
}

int pick_rc(int w) {
    for (int rc = kRowChunk; rc > 1; rc >>= 1)
        if (lds_bytes(w, rc) <= 150 * 1024) return rc;
    return 1;
}

}  // namespace

int32_t profile_grid(int64_t tiles) {
    const int64_t slots = 256;  // one workgroup per compute unit
    return (int32_t)(tiles < slots ? (tiles > 0 ? tiles : 1) : slots);
}

size_t profile_scratch_floats(int32_t grid, int32_t w) { return (size_t)grid * w * JT; }

hipError_t launch_profile(const ProfileJob &job, hipStream_t st) {
    ProfileArgs a;
    a.J = job;
    a.rc = pick_rc(job.w);
    a.cwmax = JT + job.w - 1;
    a.two_l = (float)(2.0 * job.l);
    const size_t lds = lds_bytes(job.w, a.rc);
    hipError_t e = hipFuncSetAttribute((const void *)k_profile,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_profile, dim3(job.grid), dim3(NT), lds, st, a);
    return hipGetLastError();
}

size_t profile_lds_bytes(int32_t w) { return lds_bytes(w, pick_rc(w)); }

}  // namespace pst
