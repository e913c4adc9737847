// Labelling of the series by its snippets and the per-element F1 score of
// section 5.2's accuracy experiment.  Element t takes the snippet that owns
// window min(t, n-m) (the window's nearest snippet, eq. 6); each snippet stands
// for the true class most of its elements have (ties to the lowest class);
// precision TP/(TP+FP), recall TP/(TP+FN) and F1 = 2PR/(P+R) are per true
// class (0 where a denominator is 0), summarised by their mean over the
// classes present in the truth.
#include "pst_internal.h"

namespace pst {
namespace {

constexpr int LT = 256;

// conf[p*C + c] += elements labelled by snippet p with true class c; labels
// outside [0, K) x [0, C) are counted in *bad.  Counts go through LDS when the
// table fits.
__global__ void __launch_bounds__(LT) k_confusion(LabelJob J) {
    extern __shared__ unsigned hist[];
    const int KC = J.K * J.C;
    const bool lds = J.lds;
    if (lds)
        for (int i = threadIdx.x; i < KC; i += LT) hist[i] = 0u;
    __syncthreads();
    unsigned nbad = 0;
    const int64_t Nm = J.n - J.m + 1;
    for (int64_t t = (int64_t)blockIdx.x * LT + threadIdx.x; t < J.n; t += (int64_t)gridDim.x * LT) {
        const int p = J.owner[t < Nm ? t : Nm - 1];
        const int c = J.truth[t];
        if (p < 0 || p >= J.K || c < 0 || c >= J.C) {
            ++nbad;
        } else if (lds) {
            atomicAdd(&hist[p * J.C + c], 1u);
        } else {
            atomicAdd(&J.conf[p * J.C + c], 1u);
        }
    }
    if (nbad) atomicAdd(J.bad, nbad);
    __syncthreads();
    if (lds)
        for (int i = threadIdx.x; i < KC; i += LT)
            if (hist[i]) atomicAdd(&J.conf[i], hist[i]);
}

// One block: majority map, then per-class scores and their mean.
__global__ void __launch_bounds__(LT) k_label_f1(LabelJob J) {
    __shared__ double fsum[LT];
    __shared__ int fcnt[LT];
    for (int p = threadIdx.x; p < J.K; p += LT) {
        const unsigned *row = J.conf + (size_t)p * J.C;
        int best = 0;
        for (int c = 1; c < J.C; ++c)
            if (row[c] > row[best]) best = c;
        J.map[p] = best;
    }
    __syncthreads();
    double fs = 0.0;
    int fc = 0;
    for (int c = threadIdx.x; c < J.C; c += LT) {
        uint64_t tp = 0, pred = 0, sup = 0;
        for (int p = 0; p < J.K; ++p) {
            const unsigned *row = J.conf + (size_t)p * J.C;
            sup += row[c];
            if (J.map[p] == c) {
                tp += row[c];
                for (int c2 = 0; c2 < J.C; ++c2) pred += row[c2];
            }
        }
        const double P = pred > 0 ? (double)tp / (double)pred : 0.0;
        const double Rc = sup > 0 ? (double)tp / (double)sup : 0.0;
        const double F = P + Rc > 0.0 ? 2.0 * P * Rc / (P + Rc) : 0.0;
        J.prec[c] = P;
        J.rec[c] = Rc;
        J.f1[c] = F;
        if (sup > 0) {
            fs += F;
            ++fc;
        }
    }
    fsum[threadIdx.x] = fs;
    fcnt[threadIdx.x] = fc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;  // fixed order: deterministic
        int n = 0;
        for (int i = 0; i < LT; ++i) {
            s += fsum[i];
            n += fcnt[i];
        }
        *J.macro = n > 0 ? s / n : 0.0;
    }
}

}  // namespace

hipError_t launch_label_f1(const LabelJob &job, hipStream_t st) {
    LabelJob J = job;
    const size_t kc = (size_t)J.K * J.C;
    J.lds = kc <= 8192;
    int64_t blocks = (J.n + LT - 1) / LT;
    if (blocks > 1024) blocks = 1024;
    if (blocks < 1) blocks = 1;
    hipError_t e = launch_fill_u32(J.conf, (int64_t)kc, 0u, st);
    if (e != hipSuccess) return e;
    e = launch_fill_u32(J.bad, 1, 0u, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_confusion, dim3((unsigned)blocks), dim3(LT), J.lds ? sizeof(unsigned) * kc : 0, st, J);
    hipLaunchKernelGGL(k_label_f1, dim3(1), dim3(LT), 0, st, J);
    return hipGetLastError();
}

}  // namespace pst
