// FP64 statistics of every length-l subsequence: centred means and standard
// deviations from compensated (double-double) prefix sums, plus the inverse
// norms and the two difference terms of the centred-covariance recurrence.
//
// Section 4.1 (eq. 9) evaluates the z-normalised distance matrix from dot
// products, means and standard deviations instead of normalising every
// subsequence (the technique of the paper's ref. [7]); this file produces
// those means and deviations.  Population deviation (divide by l).  A window
// whose deviation is at most 1e-6 * max(1, max|x|) is constant: its
// z-normalised form is the zero vector.
#include "pst_internal.h"

#include <math.h>

namespace pst {
namespace {

struct dd {
    double hi, lo;
};

__device__ __forceinline__ dd two_sum(double a, double b) {
    double s = a + b;
    double bb = s - a;
    double e = (a - (s - bb)) + (b - bb);
    return {s, e};
}
__device__ __forceinline__ dd renorm(double hi, double lo) {
    double s = hi + lo;
    return {s, lo - (s - hi)};
}
__device__ __forceinline__ dd dd_add(dd a, dd b) {
    dd s = two_sum(a.hi, b.hi);
    return renorm(s.hi, s.lo + (a.lo + b.lo));
}
__device__ __forceinline__ dd dd_neg(dd a) { return {-a.hi, -a.lo}; }
__device__ __forceinline__ dd two_prod(double a, double b) {
    double p = a * b;
    return {p, fma(a, b, -p)};
}
__device__ __forceinline__ dd dd_mul_d(dd a, double b) {
    dd p = two_prod(a.hi, b);
    return renorm(p.hi, p.lo + a.lo * b);
}
__device__ __forceinline__ dd dd_sqr(dd a) {
    dd p = two_prod(a.hi, a.hi);
    return renorm(p.hi, p.lo + 2.0 * a.hi * a.lo);
}

constexpr int kT = 256;
constexpr int kPer = kScanBlock / kT;  // 16 elements per thread

// Per-block sum, max |x| and a non-finite flag.
__global__ void __launch_bounds__(kT) k_reduce_part(const double *__restrict__ x, int64_t n,
                                                    double *__restrict__ part) {
    __shared__ double ssum[kT], smax[kT], sbad[kT];
    double s = 0.0, mx = 0.0, bad = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += (int64_t)gridDim.x * kT) {
        double v = x[i];
        if (!isfinite(v)) bad = 1.0;
        else {
            s += v;
            mx = fmax(mx, fabs(v));
        }
    }
    ssum[threadIdx.x] = s;
    smax[threadIdx.x] = mx;
    sbad[threadIdx.x] = bad;
    __syncthreads();
    for (int o = kT / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            ssum[threadIdx.x] += ssum[threadIdx.x + o];
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + o]);
            sbad[threadIdx.x] = fmax(sbad[threadIdx.x], sbad[threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[3 * blockIdx.x + 0] = ssum[0];
        part[3 * blockIdx.x + 1] = smax[0];
        part[3 * blockIdx.x + 2] = sbad[0];
    }
}

__global__ void k_reduce_final(const double *__restrict__ part, int np, int64_t n,
                               double *__restrict__ misc) {
    if (threadIdx.x != 0) return;
    double s = 0.0, mx = 0.0, bad = 0.0;
    for (int i = 0; i < np; ++i) {
        s += part[3 * i];
        mx = fmax(mx, part[3 * i + 1]);
        bad = fmax(bad, part[3 * i + 2]);
    }
    misc[0] = bad != 0.0 ? 0.0 : s / (double)n;
    misc[1] = mx;
    misc[2] = bad;
    misc[3] = 1e-6 * fmax(1.0, mx);
}

// Centre the series and sum each scan block: blk[b] = (sum x', sum x'^2) as dd.
__global__ void __launch_bounds__(kT) k_center_block(const double *__restrict__ x, int64_t n,
                                                     const double *__restrict__ misc,
                                                     double *__restrict__ xc,
                                                     double *__restrict__ blk) {
    __shared__ double sh[4][kT];
    const double mean = misc[0];
    int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)threadIdx.x * kPer;
    dd s{0.0, 0.0}, q{0.0, 0.0};
    for (int e = 0; e < kPer; ++e) {
        int64_t i = base + e;
        if (i < n) {
            double v = x[i] - mean;
            xc[i] = v;
            s = dd_add(s, dd{v, 0.0});
            q = dd_add(q, two_prod(v, v));
        }
    }
    sh[0][threadIdx.x] = s.hi;
    sh[1][threadIdx.x] = s.lo;
    sh[2][threadIdx.x] = q.hi;
    sh[3][threadIdx.x] = q.lo;
    __syncthreads();
    for (int o = kT / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            int t = threadIdx.x;
            dd a = dd_add(dd{sh[0][t], sh[1][t]}, dd{sh[0][t + o], sh[1][t + o]});
            dd b = dd_add(dd{sh[2][t], sh[3][t]}, dd{sh[2][t + o], sh[3][t + o]});
            sh[0][t] = a.hi;
            sh[1][t] = a.lo;
            sh[2][t] = b.hi;
            sh[3][t] = b.lo;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0)
        for (int c = 0; c < 4; ++c) blk[4 * blockIdx.x + c] = sh[c][0];
}

// Exclusive scan of the block sums (sequential; a few hundred blocks at most).
__global__ void k_scan_blocks(double *__restrict__ blk, int nb) {
    if (threadIdx.x != 0) return;
    dd s{0.0, 0.0}, q{0.0, 0.0};
    for (int b = 0; b < nb; ++b) {
        dd bs{blk[4 * b], blk[4 * b + 1]}, bq{blk[4 * b + 2], blk[4 * b + 3]};
        blk[4 * b + 0] = s.hi;
        blk[4 * b + 1] = s.lo;
        blk[4 * b + 2] = q.hi;
        blk[4 * b + 3] = q.lo;
        s = dd_add(s, bs);
        q = dd_add(q, bq);
    }
}

// Inclusive prefix sums P[i+1] = sum_{t<=i} x'_t and Q[i+1] = sum x'^2, as dd.
// pre layout: [P_hi | P_lo | Q_hi | Q_lo], each double[n+1].
__global__ void __launch_bounds__(kT) k_prefix(const double *__restrict__ xc, int64_t n,
                                               const double *__restrict__ blk,
                                               double *__restrict__ pre) {
    __shared__ double sh[4][kT];
    const int t = threadIdx.x;
    int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)t * kPer;
    dd s{0.0, 0.0}, q{0.0, 0.0};
    for (int e = 0; e < kPer; ++e) {
        int64_t i = base + e;
        if (i < n) {
            double v = xc[i];
            s = dd_add(s, dd{v, 0.0});
            q = dd_add(q, two_prod(v, v));
        }
    }
    sh[0][t] = s.hi;
    sh[1][t] = s.lo;
    sh[2][t] = q.hi;
    sh[3][t] = q.lo;
    __syncthreads();
    // Hillis-Steele inclusive scan of the per-thread totals.
    for (int o = 1; o < kT; o <<= 1) {
        dd a{sh[0][t], sh[1][t]}, b{sh[2][t], sh[3][t]};
        if (t >= o) {
            a = dd_add(a, dd{sh[0][t - o], sh[1][t - o]});
            b = dd_add(b, dd{sh[2][t - o], sh[3][t - o]});
        }
        __syncthreads();
        sh[0][t] = a.hi;
        sh[1][t] = a.lo;
        sh[2][t] = b.hi;
        sh[3][t] = b.lo;
        __syncthreads();
    }
    dd offs{blk[4 * blockIdx.x], blk[4 * blockIdx.x + 1]};
    dd offq{blk[4 * blockIdx.x + 2], blk[4 * blockIdx.x + 3]};
    if (t > 0) {
        offs = dd_add(offs, dd{sh[0][t - 1], sh[1][t - 1]});
        offq = dd_add(offq, dd{sh[2][t - 1], sh[3][t - 1]});
    }
    const int64_t N1 = n + 1;
    double *Ph = pre, *Pl = pre + N1, *Qh = pre + 2 * N1, *Ql = pre + 3 * N1;
    if (blockIdx.x == 0 && t == 0) {
        Ph[0] = 0.0;
        Pl[0] = 0.0;
        Qh[0] = 0.0;
        Ql[0] = 0.0;
    }
    for (int e = 0; e < kPer; ++e) {
        int64_t i = base + e;
        if (i < n) {
            double v = xc[i];
            offs = dd_add(offs, dd{v, 0.0});
            offq = dd_add(offq, two_prod(v, v));
            Ph[i + 1] = offs.hi;
            Pl[i + 1] = offs.lo;
            Qh[i + 1] = offq.hi;
            Ql[i + 1] = offq.lo;
        }
    }
}

__device__ __forceinline__ dd pre_at(const double *h, const double *lo, int64_t i) {
    return dd{h[i], lo[i]};
}

// Window statistics from the prefix sums.
__global__ void __launch_bounds__(kT) k_winstats(const double *__restrict__ xc, int64_t n, int l,
                                                 const double *__restrict__ pre,
                                                 const double *__restrict__ misc,
                                                 double *__restrict__ mu, float *__restrict__ inv,
                                                 float *__restrict__ hh, float *__restrict__ df,
                                                 float *__restrict__ dg, double *__restrict__ xpad) {
    const int64_t Nl = n - l + 1;
    const int64_t N1 = n + 1;
    const double *Ph = pre, *Pl = pre + N1, *Qh = pre + 2 * N1, *Ql = pre + 3 * N1;
    const double thr = misc[3];
    const double dl = (double)l;
    for (int64_t j = (int64_t)blockIdx.x * kT + threadIdx.x; j < Nl + kStatsPad; j += (int64_t)gridDim.x * kT) {
        if (j >= Nl) {  // zeroed padding: readers may run a few windows past the end
            mu[j] = 0.0;
            inv[j] = 0.0f;
            hh[j] = 0.0f;
            df[j] = 0.0f;
            dg[j] = 0.0f;
            xpad[j - Nl] = 0.0;
            continue;
        }
        dd S = dd_add(pre_at(Ph, Pl, j + l), dd_neg(pre_at(Ph, Pl, j)));
        dd Q = dd_add(pre_at(Qh, Ql, j + l), dd_neg(pre_at(Qh, Ql, j)));
        // l^2 var = l * Q - S^2, in double-double
        dd v2 = dd_add(dd_mul_d(Q, dl), dd_neg(dd_sqr(S)));
        double var = (v2.hi + v2.lo) / (dl * dl);
        double sig = sqrt(fmax(var, 0.0));
        double m0 = (S.hi + S.lo) / dl;
        mu[j] = m0;
        bool cst = !(sig > thr);
        inv[j] = cst ? 0.0f : (float)(1.0 / (sig * sqrt(dl)));
        hh[j] = cst ? 0.5f : 0.0f;
        if (j + 1 < Nl) {
            dd S1 = dd_add(pre_at(Ph, Pl, j + 1 + l), dd_neg(pre_at(Ph, Pl, j + 1)));
            double m1 = (S1.hi + S1.lo) / dl;
            df[j] = (float)((xc[j + l] - xc[j]) * 0.5);
            dg[j] = (float)((xc[j + l] - m1) + (xc[j] - m0));
        } else {
            df[j] = 0.0f;
            dg[j] = 0.0f;
        }
    }
}

inline size_t al(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

StatsLayout stats_layout(int64_t len, int32_t l) {
    StatsLayout L{};
    L.len = len;
    L.l = l;
    L.Nl = len - l + 1;
    L.nblk = (int32_t)((len + kScanBlock - 1) / kScanBlock);
    size_t o = 0;
    L.xc = o;   o = al(o + sizeof(double) * (len + kStatsPad));
    L.mu = o;   o = al(o + sizeof(double) * (L.Nl + kStatsPad));
    L.inv = o;  o = al(o + sizeof(float) * (L.Nl + kStatsPad));
    L.h = o;    o = al(o + sizeof(float) * (L.Nl + kStatsPad));
    L.df = o;   o = al(o + sizeof(float) * (L.Nl + kStatsPad));
    L.dg = o;   o = al(o + sizeof(float) * (L.Nl + kStatsPad));
    L.pre = o;  o = al(o + sizeof(double) * 4 * (len + 1));
    L.blk = o;  o = al(o + sizeof(double) * 4 * L.nblk);
    L.part = o; o = al(o + sizeof(double) * 3 * 1024);
    L.misc = o; o = al(o + sizeof(double) * 8);
    L.total = o;
    return L;
}

Stats stats_view(char *base, const StatsLayout &L) {
    Stats s;
    s.xc = (const double *)(base + L.xc);
    s.mu = (const double *)(base + L.mu);
    s.inv = (const float *)(base + L.inv);
    s.h = (const float *)(base + L.h);
    s.df = (const float *)(base + L.df);
    s.dg = (const float *)(base + L.dg);
    return s;
}

hipError_t launch_series_stats(const double *x, char *base, const StatsLayout &L, hipStream_t st) {
    const int64_t n = L.len;
    double *part = (double *)(base + L.part);
    double *misc = (double *)(base + L.misc);
    double *xc = (double *)(base + L.xc);
    double *blk = (double *)(base + L.blk);
    double *pre = (double *)(base + L.pre);
    int np = (int)std::min<int64_t>(1024, (n + kT * 16 - 1) / (kT * 16));
    if (np < 1) np = 1;
    hipLaunchKernelGGL(k_reduce_part, dim3(np), dim3(kT), 0, st, x, n, part);
    hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(64), 0, st, part, np, n, misc);
    hipLaunchKernelGGL(k_center_block, dim3(L.nblk), dim3(kT), 0, st, x, n, misc, xc, blk);
    hipLaunchKernelGGL(k_scan_blocks, dim3(1), dim3(64), 0, st, blk, L.nblk);
    hipLaunchKernelGGL(k_prefix, dim3(L.nblk), dim3(kT), 0, st, xc, n, blk, pre);
    int nw = (int)std::min<int64_t>(4096, (L.Nl + kStatsPad + kT - 1) / kT);
    if (nw < 1) nw = 1;
    hipLaunchKernelGGL(k_winstats, dim3(nw), dim3(kT), 0, st, xc, n, L.l, pre, misc,
                       (double *)(base + L.mu), (float *)(base + L.inv), (float *)(base + L.h),
                       (float *)(base + L.df), (float *)(base + L.dg), xc + n);
    return hipGetLastError();
}

}  // namespace pst
