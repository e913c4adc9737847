// Snippet selection on the profile set D, entirely on device.
//
//   - greedy minimum-area search (section 4.1, eqs. 16-17): K rounds; in each,
//     every unchosen segment's area sum_j min(M_j, D_s(j)) is summed in FP64 in
//     a fixed order (per-block tree sums, then blocks in order), the smallest
//     area wins with ties to the lowest segment index, and M <- min(M, D_pick);
//   - neighbours and frac (eqs. 6-7): each window is owned by the chosen
//     snippet with the smallest profile value there, ties to the earlier pick;
//   - the snippet-length criterion numerator (eq. 18): sum over ordered pairs
//     of picked profiles of sum_j |D_p(j) - D_q(j)|.
#include "pst_internal.h"

#include <math.h>

namespace pst {
namespace {

constexpr int GT = 256;

__global__ void k_set_u32(uint32_t *__restrict__ p, int64_t n, uint32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * GT + threadIdx.x; i < n; i += (int64_t)gridDim.x * GT)
        p[i] = v;
}

__device__ __forceinline__ double block_sum(double v, double *red) {
    const int t = threadIdx.x;
    red[t] = v;
    __syncthreads();
    for (int o = GT / 2; o > 0; o >>= 1) {
        if (t < o) red[t] += red[t + o];
        __syncthreads();
    }
    double r = red[0];
    __syncthreads();
    return r;
}

// Greedy jobs of one launch: the grid's last dimension picks the job.
struct GreedyBatch {
    GreedyJob J[kMaxJobs];
    int64_t part_end[kMaxJobs];  // job j owns area blocks [part_end[j-1], part_end[j])
    int32_t n, kmax;
};
static_assert(sizeof(GreedyBatch) <= 4000, "kernel arguments must fit the 4 KB limit");

// M = +inf and nothing chosen, for job blockIdx.y.
__global__ void k_greedy_init(GreedyBatch B) {
    const GreedyJob &g = B.J[blockIdx.y];
    for (int64_t i = (int64_t)blockIdx.x * GT + threadIdx.x; i < g.Nm; i += (int64_t)gridDim.x * GT)
        g.M[i] = INFINITY;
    for (int64_t i = (int64_t)blockIdx.x * GT + threadIdx.x; i < g.nseg; i += (int64_t)gridDim.x * GT)
        g.chosen[i] = 0;
}

// part[s * nblk + b] = sum over block b's windows of min(M_j, D_s(j)), one
// workgroup per (job, segment, block), in round iter (jobs with fewer rounds
// skip; iter < 0: no round check).
__global__ void __launch_bounds__(GT) k_area_part(GreedyBatch B, int iter) {
    __shared__ double red[GT];
    int jb = 0;
    while (jb + 1 < B.n && (int64_t)blockIdx.x >= B.part_end[jb]) ++jb;
    const GreedyJob &g = B.J[jb];
    const int64_t local = (int64_t)blockIdx.x - (jb ? B.part_end[jb - 1] : 0);
    const int s = (int)(local / g.nblk), b = (int)(local - (int64_t)s * g.nblk);
    if (iter >= 0 && iter >= g.K) return;
    if (g.chosen[s]) return;
    const int64_t j0 = (int64_t)b * kSumBlock;
    const int64_t j1 = j0 + kSumBlock < g.Nm ? j0 + kSumBlock : g.Nm;
    const float *Ds = g.D + (int64_t)s * g.ld;
    double acc = 0.0;
    for (int64_t j = j0 + threadIdx.x; j < j1; j += GT) acc += (double)fminf(g.M[j], Ds[j]);
    double tot = block_sum(acc, red);
    if (threadIdx.x == 0) g.part[(int64_t)s * g.nblk + b] = tot;
}

// One block per job: smallest area among unchosen segments, ties to the
// lowest index.
__global__ void __launch_bounds__(1024) k_pick(GreedyBatch B, int iter) {
    __shared__ double ra[1024];
    __shared__ int rs[1024];
    const GreedyJob &g = B.J[blockIdx.x];
    if (iter >= g.K) return;
    const int t = threadIdx.x;
    double best = INFINITY;
    int bs = 0x7fffffff;
    for (int s = t; s < g.nseg; s += 1024) {
        if (g.chosen[s]) continue;
        double a = 0.0;
        const double *p = g.part + (int64_t)s * g.nblk;
        for (int b = 0; b < g.nblk; ++b) a += p[b];
        if (a < best || (a == best && s < bs)) {
            best = a;
            bs = s;
        }
    }
    ra[t] = best;
    rs[t] = bs;
    __syncthreads();
    for (int o = 512; o > 0; o >>= 1) {
        if (t < o) {
            const double a2 = ra[t + o];
            const int s2 = rs[t + o];
            if (a2 < ra[t] || (a2 == ra[t] && s2 < rs[t])) {
                ra[t] = a2;
                rs[t] = s2;
            }
        }
        __syncthreads();
    }
    if (t == 0) {
        g.pick[iter] = rs[0];
        g.area[iter] = ra[0];
        g.chosen[rs[0]] = 1;
    }
}

__global__ void k_update_M(GreedyBatch B, int iter) {
    const GreedyJob &g = B.J[blockIdx.y];
    if (iter >= g.K) return;
    const float *Dp = g.D + (int64_t)g.pick[iter] * g.ld;
    for (int64_t j = (int64_t)blockIdx.x * GT + threadIdx.x; j < g.Nm; j += (int64_t)gridDim.x * GT)
        g.M[j] = fminf(g.M[j], Dp[j]);
}

__global__ void k_zero_counts(GreedyBatch B) {
    const GreedyJob &g = B.J[blockIdx.y];
    for (int64_t i = (int64_t)blockIdx.x * GT + threadIdx.x; i < g.K; i += (int64_t)gridDim.x * GT) g.count[i] = 0;
}

__global__ void __launch_bounds__(GT) k_owner(GreedyBatch B) {
    extern __shared__ int cnt_lds[];
    const GreedyJob &g = B.J[blockIdx.y];
    const bool use_lds = B.kmax <= 1024;  // the launch sized LDS for every job's counts
    if (use_lds) {
        for (int p = threadIdx.x; p < g.K; p += GT) cnt_lds[p] = 0;
        __syncthreads();
    }
    for (int64_t j = (int64_t)blockIdx.x * GT + threadIdx.x; j < g.Nm; j += (int64_t)gridDim.x * GT) {
        float best = g.D[(int64_t)g.pick[0] * g.ld + j];
        int bp = 0;
        for (int p = 1; p < g.K; ++p) {
            const float v = g.D[(int64_t)g.pick[p] * g.ld + j];
            if (v < best) {
                best = v;
                bp = p;
            }
        }
        if (g.owner) g.owner[j] = bp;
        if (use_lds) atomicAdd(&cnt_lds[bp], 1);
        else atomicAdd(&g.count[bp], 1);
        if (g.profiles)
            for (int p = 0; p < g.K; ++p)
                g.profiles[(int64_t)p * g.Nm + j] = g.D[(int64_t)g.pick[p] * g.ld + j];
    }
    if (use_lds) {
        __syncthreads();
        for (int p = threadIdx.x; p < g.K; p += GT)
            if (cnt_lds[p]) atomicAdd(&g.count[p], cnt_lds[p]);
    }
}

__global__ void __launch_bounds__(GT) k_crit_part(GreedyJob g) {
    __shared__ double red[GT];
    double acc = 0.0;
    for (int64_t j = (int64_t)blockIdx.x * GT + threadIdx.x; j < g.Nm; j += (int64_t)gridDim.x * GT) {
        for (int p = 0; p < g.K; ++p) {
            const float a = g.D[(int64_t)g.pick[p] * g.ld + j];
            for (int q = p + 1; q < g.K; ++q)
                acc += fabs((double)a - (double)g.D[(int64_t)g.pick[q] * g.ld + j]);
        }
    }
    double tot = block_sum(acc, red);
    if (threadIdx.x == 0) g.crit[blockIdx.x] = tot;
}

__global__ void k_crit_final(GreedyJob g) {
    if (threadIdx.x != 0) return;
    double s = 0.0;
    for (int b = 0; b < g.nblk2; ++b) s += g.crit[b];
    g.crit[g.nblk2] = 2.0 * s;  // ordered pairs p != q
}

__global__ void k_gather(SweepGather G) {
    const int stride = 3 + 3 * G.K;
    for (int i = threadIdx.x; i < G.nm * stride; i += blockDim.x) {
        const int c = i / stride, e = i - c * stride;
        double v;
        if (e == 0) v = *G.crit[c];
        else if (e == 1) v = (double)*G.dmax[c];
        else if (e == 2) v = *G.bad[c];
        else if (e < 3 + G.K) v = G.area[c][e - 3];
        else if (e < 3 + 2 * G.K) v = (double)G.pick[c][e - 3 - G.K];
        else v = (double)G.count[c][e - 3 - 2 * G.K];
        G.out[i] = v;
    }
}

// One block per request of a served batch (see ResultPack).
__global__ void k_pack_results(ResultPack P) {
    const int i = blockIdx.x, K = P.K[i];
    double *h = P.out + P.off[i];
    for (int t = threadIdx.x; t < 4; t += blockDim.x) h[t] = P.misc[i][t];
    int32_t *hp = (int32_t *)(h + 4), *hc = (int32_t *)(h + 4 + 2 * K);
    for (int t = threadIdx.x; t < K; t += blockDim.x) {
        hp[t] = P.pick[i][t];
        h[4 + K + t] = P.area[i][t];
        hc[t] = P.count[i][t];
    }
    if (threadIdx.x == 0) *(uint32_t *)(h + 4 + 3 * K) = *P.dmax[i];
}

inline int grid_for(int64_t n) {
    int64_t b = (n + GT - 1) / GT;
    return (int)(b < 2048 ? (b > 0 ? b : 1) : 2048);
}

}  // namespace

hipError_t launch_fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t st) {
    hipLaunchKernelGGL(k_set_u32, dim3(grid_for(n)), dim3(GT), 0, st, p, n, v);
    return hipGetLastError();
}

namespace {
GreedyBatch batch_of(const GreedyJob *g, int n) {
    GreedyBatch B{};
    B.n = n;
    int64_t acc = 0;
    for (int i = 0; i < n; ++i) {
        B.J[i] = g[i];
        acc += (int64_t)g[i].nseg * g[i].nblk;
        B.part_end[i] = acc;
        B.kmax = g[i].K > B.kmax ? g[i].K : B.kmax;
    }
    return B;
}
}  // namespace

hipError_t launch_greedy_init(const GreedyJob &g, hipStream_t st) {
    const GreedyBatch B = batch_of(&g, 1);
    hipLaunchKernelGGL(k_greedy_init, dim3(grid_for(g.Nm > g.nseg ? g.Nm : g.nseg), 1), dim3(GT), 0, st, B);
    return hipGetLastError();
}

hipError_t launch_greedy_batch(const GreedyJob *g, int n, hipStream_t st) {
    if (n < 1 || n > kMaxJobs) return hipErrorInvalidValue;
    const GreedyBatch B = batch_of(g, n);
    int64_t span = 0;
    for (int i = 0; i < n; ++i) {
        span = g[i].Nm > span ? g[i].Nm : span;
        span = g[i].nseg > span ? g[i].nseg : span;
    }
    const int64_t parts = B.part_end[n - 1];
    if (parts < 1 || parts > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_greedy_init, dim3(grid_for(span), n), dim3(GT), 0, st, B);
    for (int it = 0; it < B.kmax; ++it) {
        hipLaunchKernelGGL(k_area_part, dim3((unsigned)parts), dim3(GT), 0, st, B, it);
        hipLaunchKernelGGL(k_pick, dim3(n), dim3(1024), 0, st, B, it);
        hipLaunchKernelGGL(k_update_M, dim3(grid_for(span), n), dim3(GT), 0, st, B, it);
    }
    return hipGetLastError();
}

hipError_t launch_greedy(const GreedyJob &g, hipStream_t st) { return launch_greedy_batch(&g, 1, st); }

hipError_t launch_area_parts(const GreedyJob &g, hipStream_t st) {
    hipLaunchKernelGGL(k_area_part, dim3((unsigned)((int64_t)g.nseg * g.nblk)), dim3(GT), 0, st, batch_of(&g, 1),
                       -1);
    return hipGetLastError();
}

hipError_t launch_pick(const GreedyJob &g, int iter, hipStream_t st) {
    hipLaunchKernelGGL(k_pick, dim3(1), dim3(1024), 0, st, batch_of(&g, 1), iter);
    return hipGetLastError();
}

hipError_t launch_update_M(const GreedyJob &g, int iter, hipStream_t st) {
    hipLaunchKernelGGL(k_update_M, dim3(grid_for(g.Nm), 1), dim3(GT), 0, st, batch_of(&g, 1), iter);
    return hipGetLastError();
}

hipError_t launch_owner_batch(const GreedyJob *g, int n, hipStream_t st) {
    if (n < 1 || n > kMaxJobs) return hipErrorInvalidValue;
    const GreedyBatch B = batch_of(g, n);
    int64_t Nm = 1;
    for (int i = 0; i < n; ++i) Nm = g[i].Nm > Nm ? g[i].Nm : Nm;
    const int K = B.kmax > 1 ? B.kmax : 1;
    hipLaunchKernelGGL(k_zero_counts, dim3(grid_for(K), n), dim3(GT), 0, st, B);
    const size_t lds = K <= 1024 ? sizeof(int) * K : 0;
    hipLaunchKernelGGL(k_owner, dim3(grid_for(Nm), n), dim3(GT), lds, st, B);
    return hipGetLastError();
}

hipError_t launch_owner(const GreedyJob &g, hipStream_t st) { return launch_owner_batch(&g, 1, st); }

hipError_t launch_pack_results(const ResultPack &r, hipStream_t st) {
    if (r.n < 1 || r.n > kMaxJobs) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_pack_results, dim3(r.n), dim3(64), 0, st, r);
    return hipGetLastError();
}

hipError_t launch_gather(const SweepGather &g, hipStream_t st) {
    hipLaunchKernelGGL(k_gather, dim3(1), dim3(256), 0, st, g);
    return hipGetLastError();
}

hipError_t launch_criterion(const GreedyJob &g, hipStream_t st) {
    hipLaunchKernelGGL(k_crit_part, dim3(g.nblk2), dim3(GT), 0, st, g);
    hipLaunchKernelGGL(k_crit_final, dim3(1), dim3(64), 0, st, g);
    return hipGetLastError();
}

}  // namespace pst
