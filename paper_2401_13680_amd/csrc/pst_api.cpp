// Host runtime behind include/pst.h: argument validation, workspace layout,
// launch sequencing on the caller's stream, and the host-side tail of the
// snippet search (ordering K records by frac, eq. 8).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <functional>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "../../include/pst.h"
#include "pst_internal.h"
#include "pst_sched.h"

struct GraphEntry {
    std::vector<int64_t> key;
    hipGraphExec_t exec;
};

struct pst_ctx {
    int device;
    hipStream_t stream;
    hipStream_t cap;              // private stream for graph capture (lazily created)
    bool poisoned;
    bool timing;
    bool timed;
    hipEvent_t ev0, ev1;
    void *fixed_scratch;          // device address of the fixed scratch on this device (or null)
    // options (pst_set_option)
    int opt_graph = 1, opt_autotune = 0, opt_grid = 0, opt_dynamic = 1, opt_batched = 1, opt_anchor = 0;
    int opt_tune_geometry = 0, opt_one_launch = 0;
    std::vector<GraphEntry> graphs;
    char err[512];
};

namespace {

using namespace pst;

size_t al(size_t v) { return (v + 255) & ~(size_t)255; }

int fail(pst_ctx *c, int code, const char *fmt, ...) {
    if (c) {
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(c->err, sizeof c->err, fmt, ap);
        va_end(ap);
        if (code == PST_EDEVICE) c->poisoned = true;
    }
    return code;
}

#define HIPCHK(ctx, expr)                                                                  \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(ctx, PST_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));  \
    } while (0)

struct Layout {
    int64_t n, Nl, Nm;
    int32_t m, l, w, k, K, nseg;
    int64_t ntile;
    int32_t grid, nblk, nblk2;
    StatsLayout sT, sQ;
    size_t o_T, o_Q, o_rw, o_D, o_M, o_part, o_pick, o_area, o_chosen, o_count, o_crit, o_dmax;
    size_t total;
};

int32_t eff_k(int32_t k, int32_t m) { return k > 0 ? k : (m + 9) / 10; }

// Validate sizes; on success fill the layout.  K == 0 means "no snippets".
// Without with_rw the profile kernel's scratch is left out (a batch that
// shares one scratch region supplies it).
int plan(pst_ctx *c, int64_t n, int32_t m, int32_t l, int32_t k, int32_t K, Layout *L, bool with_rw = true) {
    if (m < 2 || n < m) return fail(c, PST_EINVAL, "need 2 <= m <= n (m=%d, n=%lld)", m, (long long)n);
    if (l < 2 || l > m) return fail(c, PST_EINVAL, "need 2 <= l <= m (l=%d, m=%d)", l, m);
    const int32_t w = m - l + 1;
    if (w > kMaxW) return fail(c, PST_EINVAL, "w = m-l+1 = %d exceeds %d", w, kMaxW);
    if (n > (int64_t)1 << 31) return fail(c, PST_EINVAL, "n too large");
    const int64_t nseg = n / m;
    if (K < 0 || K > nseg) return fail(c, PST_EINVAL, "need 1 <= K <= n/m (K=%d, n/m=%lld)", K, (long long)nseg);
    L->n = n;
    L->m = m;
    L->l = l;
    L->w = w;
    L->k = eff_k(k, m);
    L->K = K;
    L->nseg = (int32_t)nseg;
    L->Nl = n - l + 1;
    L->Nm = n - m + 1;
    L->ntile = (L->Nm + profile_tile_windows(w) - 1) / profile_tile_windows(w);
    L->grid = profile_grid(L->ntile * nseg, w);
    L->nblk = (int32_t)((L->Nm + kSumBlock - 1) / kSumBlock);
    L->nblk2 = (int32_t)std::min<int64_t>(1024, (L->Nm + 255) / 256);
    L->sT = stats_layout(n, l);
    L->sQ = stats_layout(m, l);
    size_t o = 0;
    L->o_T = o;      o = al(o + L->sT.total);
    L->o_Q = o;      o = al(o + L->sQ.total);
    L->o_rw = o;     o = al(o + (with_rw ? sizeof(float) * profile_scratch_bound(L->Nm, nseg, w) : 0));
    L->o_D = o;      o = al(o + sizeof(float) * (size_t)nseg * L->Nm);
    L->o_M = o;      o = al(o + sizeof(float) * L->Nm);
    L->o_part = o;   o = al(o + sizeof(double) * (size_t)nseg * L->nblk);
    L->o_pick = o;   o = al(o + sizeof(int32_t) * std::max(K, 1));
    L->o_area = o;   o = al(o + sizeof(double) * std::max(K, 1));
    L->o_chosen = o; o = al(o + (size_t)nseg);
    L->o_count = o;  o = al(o + sizeof(int32_t) * std::max(K, 1));
    L->o_crit = o;   o = al(o + sizeof(double) * (L->nblk2 + 1));
    L->o_dmax = o;   o = al(o + 256);
    L->total = o;
    return PST_OK;
}

int begin(pst_ctx *c) {
    if (!c) return PST_EINVAL;
    if (c->poisoned) return PST_EDEVICE;
    c->err[0] = 0;
    HIPCHK(c, hipSetDevice(c->device));
    return PST_OK;
}

int check_ws(pst_ctx *c, const Layout &L, void *ws, size_t ws_bytes) {
    if (!ws) return fail(c, PST_EINVAL, "workspace is NULL");
    if (((uintptr_t)ws & 255) != 0) return fail(c, PST_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < L.total)
        return fail(c, PST_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, L.total);
    return PST_OK;
}

// Statistics of a series; reports non-finite input (one stream sync).
int series_stats(pst_ctx *c, const double *x, char *base, const StatsLayout &SL, const char *what) {
    HIPCHK(c, launch_series_stats(x, base, SL, c->stream));
    double misc[4];
    HIPCHK(c, hipMemcpyAsync(misc, stats_misc(base, SL), sizeof misc, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (misc[2] != 0.0) return fail(c, PST_EINVAL, "%s holds a non-finite value", what);
    return PST_OK;
}

// Launch the profile kernel, bracketed by the context's events when timing.
hipError_t timed_profile(pst_ctx *c, ProfileJob j) {
    j.anchor_every = c->opt_anchor;
    if (c->timing) {
        hipError_t e = hipEventRecord(c->ev0, c->stream);
        if (e != hipSuccess) return e;
    }
    hipError_t e = launch_profile(j, c->stream);
    if (e != hipSuccess) {
        fprintf(stderr, "pst: profile launch failed (w=%d grid=%d lds=%zu): %s\n", j.w, j.grid,
                profile_lds_bytes(j.w), hipGetErrorString(e));
        return e;
    }
    if (c->timing) {
        e = hipEventRecord(c->ev1, c->stream);
        if (e != hipSuccess) return e;
        c->timed = true;
    }
    return hipSuccess;
}

ProfileJob job_for(const Layout &L, char *ws, float *D, int64_t ld, unsigned *dmax_bits) {
    ProfileJob j{};
    j.col = stats_view(ws + L.o_T, L.sT);
    j.row = j.col;
    j.row_stride = L.m;
    j.n = L.n;
    j.Nl = L.Nl;
    j.Nm = L.Nm;
    j.m = L.m;
    j.l = L.l;
    j.w = L.w;
    j.k = L.k;
    j.nq = L.nseg;
    j.D = D;
    j.ld = ld;
    j.rw = (float *)(ws + L.o_rw);
    j.dmax_bits = dmax_bits;
    j.grid = L.grid;
    return j;
}

GreedyJob greedy_for(const Layout &L, char *ws, const float *D, int64_t ld) {
    GreedyJob g{};
    g.D = D;
    g.ld = ld;
    g.Nm = L.Nm;
    g.nseg = L.nseg;
    g.K = L.K;
    g.M = (float *)(ws + L.o_M);
    g.part = (double *)(ws + L.o_part);
    g.nblk = L.nblk;
    g.pick = (int32_t *)(ws + L.o_pick);
    g.area = (double *)(ws + L.o_area);
    g.chosen = (uint8_t *)(ws + L.o_chosen);
    g.count = (int32_t *)(ws + L.o_count);
    g.crit = (double *)(ws + L.o_crit);
    g.nblk2 = L.nblk2;
    return g;
}

// D of all segments into ws (ld = Nm), then the greedy search and neighbours.
// Leaves picks, areas, counts and dmax in ws; no host sync.
int snippets_device(pst_ctx *c, const double *T, const Layout &L, char *ws, int32_t *owner,
                    float *profiles, bool with_criterion) {
    int rc = series_stats(c, T, ws + L.o_T, L.sT, "T");
    if (rc) return rc;
    unsigned *dmax = (unsigned *)(ws + L.o_dmax);
    HIPCHK(c, launch_fill_u32(dmax, 1, 0u, c->stream));
    float *D = (float *)(ws + L.o_D);
    HIPCHK(c, timed_profile(c, job_for(L, ws, D, L.Nm, dmax)));
    GreedyJob g = greedy_for(L, ws, D, L.Nm);
    g.owner = owner;
    g.profiles = profiles;
    HIPCHK(c, launch_greedy(g, c->stream));
    HIPCHK(c, launch_owner(g, c->stream));
    if (with_criterion) HIPCHK(c, launch_criterion(g, c->stream));
    return PST_OK;
}

int collect_records(pst_ctx *c, const Layout &L, char *ws, pst_snippet *out, float *dmax_host,
                    double *crit_host) {
    std::vector<int32_t> pick(L.K), cnt(L.K);
    std::vector<double> area(L.K);
    unsigned dbits = 0;
    double crit = 0.0;
    HIPCHK(c, hipMemcpyAsync(pick.data(), ws + L.o_pick, sizeof(int32_t) * L.K, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(cnt.data(), ws + L.o_count, sizeof(int32_t) * L.K, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(area.data(), ws + L.o_area, sizeof(double) * L.K, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipMemcpyAsync(&dbits, ws + L.o_dmax, sizeof dbits, hipMemcpyDeviceToHost, c->stream));
    if (crit_host)
        HIPCHK(c, hipMemcpyAsync(&crit, ws + L.o_crit + sizeof(double) * L.nblk2, sizeof crit,
                                 hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    std::vector<pst_snippet> rec(L.K);
    for (int p = 0; p < L.K; ++p) {
        rec[p].segment = pick[p];
        rec[p].greedy_rank = p;
        rec[p].frac = (double)cnt[p] / (double)L.Nm;
        rec[p].area_after = area[p];
    }
    std::stable_sort(rec.begin(), rec.end(),
                     [](const pst_snippet &a, const pst_snippet &b) { return a.frac > b.frac; });
    if (out) std::memcpy(out, rec.data(), sizeof(pst_snippet) * L.K);
    float dmax;
    std::memcpy(&dmax, &dbits, sizeof dmax);
    if (dmax_host) *dmax_host = dmax;
    if (crit_host) *crit_host = dmax > 0.0f ? crit / (double)dmax : 0.0;
    return PST_OK;
}


// ---------------------------------------------------------------- multivariate
// The snippet search runs on each coordinate of a d-dimensional series on its
// own (section 3.2, over the coordinates of eqs. 1-2): one profile job per
// coordinate, all of them in one persistent launch over a shared scratch
// region, then each coordinate's greedy search and neighbours.
struct MultiPlan {
    Layout L;          // one coordinate's region (without profile scratch)
    int32_t d = 0, grid = 0;
    size_t o_rw = 0, o_counter = 0, total = 0;
};

int plan_multi(pst_ctx *c, int32_t d, int64_t n, int32_t m, int32_t l, int32_t k, int32_t K, MultiPlan *P) {
    if (d < 1 || d > kMaxJobs) return fail(c, PST_EINVAL, "need 1 <= d <= %d coordinates (d=%d)", kMaxJobs, d);
    if (K < 1) return fail(c, PST_EINVAL, "need K >= 1 (K=%d)", K);
    const int rc = plan(c, n, m, l, k, K, &P->L, false);
    if (rc) return rc;
    P->d = d;
    P->grid = profile_grid(P->L.ntile * P->L.nseg * d, P->L.w);
    size_t o = (size_t)d * P->L.total;
    P->o_rw = o;       o = al(o + sizeof(float) * profile_scratch_bound(P->L.Nm, (int64_t)P->L.nseg * d, P->L.w));
    P->o_counter = o;  o = al(o + 256);
    P->total = o;
    return PST_OK;
}

int run_multi(pst_ctx *c, const MultiPlan &P, const double *T, int64_t ldT, char *ws, pst_snippet *out,
              int32_t *owner, float *dmax_host) {
    const Layout &L = P.L;
    auto region = [&](int j) { return ws + (size_t)j * L.total; };
    // statistics of every coordinate; one sync for the finiteness checks
    std::vector<double> misc((size_t)P.d * 4);
    for (int j = 0; j < P.d; ++j) {
        HIPCHK(c, launch_series_stats(T + (size_t)j * ldT, region(j) + L.o_T, L.sT, c->stream));
        HIPCHK(c, hipMemcpyAsync(&misc[(size_t)j * 4], stats_misc(region(j) + L.o_T, L.sT), 4 * sizeof(double),
                                 hipMemcpyDeviceToHost, c->stream));
    }
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int j = 0; j < P.d; ++j)
        if (misc[(size_t)j * 4 + 2] != 0.0) return fail(c, PST_EINVAL, "coordinate %d holds a non-finite value", j);
    ProfileJob jobs[kMaxJobs];
    for (int j = 0; j < P.d; ++j) {
        unsigned *dm = (unsigned *)(region(j) + L.o_dmax);
        HIPCHK(c, launch_fill_u32(dm, 1, 0u, c->stream));
        jobs[j] = job_for(L, region(j), (float *)(region(j) + L.o_D), L.Nm, dm);
        jobs[j].rw = (float *)(ws + P.o_rw);
        jobs[j].grid = P.grid;
        jobs[j].anchor_every = c->opt_anchor;
    }
    uint32_t *counter = (uint32_t *)(ws + P.o_counter);
    HIPCHK(c, launch_fill_u32(counter, 1, 0u, c->stream));
    HIPCHK(c, profile_prepare(L.w));
    if (c->timing) HIPCHK(c, hipEventRecord(c->ev0, c->stream));
    HIPCHK(c, launch_profile_batch(jobs, P.d, P.grid, counter, c->stream));
    if (c->timing) {
        HIPCHK(c, hipEventRecord(c->ev1, c->stream));
        c->timed = true;
    }
    // every coordinate's greedy search and neighbours in the same launches
    for (int j0 = 0; j0 < P.d; j0 += kMaxJobs) {
        GreedyJob gs[kMaxJobs];
        const int nj = std::min(kMaxJobs, P.d - j0);
        for (int i = 0; i < nj; ++i) {
            const int j = j0 + i;
            gs[i] = greedy_for(L, region(j), (const float *)(region(j) + L.o_D), L.Nm);
            gs[i].owner = owner ? owner + (size_t)j * L.Nm : nullptr;
            gs[i].profiles = nullptr;
        }
        HIPCHK(c, launch_greedy_batch(gs, nj, c->stream));
        HIPCHK(c, launch_owner_batch(gs, nj, c->stream));
    }
    for (int j = 0; j < P.d; ++j) {
        const int rc = collect_records(c, L, region(j), out + (size_t)j * L.K, dmax_host ? dmax_host + j : nullptr,
                                       nullptr);
        if (rc) return rc;
    }
    return PST_OK;
}

// ---------------------------------------------------------------- bounded memory
// The profile set D never held whole: every greedy round recomputes D in
// blocks of B segments, reduces each block to the segments' areas against the
// current curve M (eq. 17) and drops it; the picked segment's profile is then
// recomputed alone, kept (K rows) and folded into M.  Device memory is
// O(B (n-m+1) + K (n-m+1)) instead of O(nseg (n-m+1)), for K+1 times the
// profile work.  A cell's arithmetic does not depend on the block it is
// computed in, so every step sees the same values as the in-core path.
struct BlockedLayout {
    Layout L;            // sizes (its D and scratch regions are not used)
    int32_t B = 0, grid = 0;
    size_t o_T, o_Dblk, o_P, o_M, o_part, o_pick, o_area, o_chosen, o_count, o_iota, o_dmax, o_crit, o_rw, total;
};

int plan_blocked(pst_ctx *c, int64_t n, int32_t m, int32_t l, int32_t k, int32_t K, int32_t B, BlockedLayout *P) {
    if (K < 1) return fail(c, PST_EINVAL, "need K >= 1 (K=%d)", K);
    int rc = plan(c, n, m, l, k, K, &P->L, false);
    if (rc) return rc;
    const Layout &L = P->L;
    if (B < 1 || B > L.nseg) return fail(c, PST_EINVAL, "need 1 <= seg_block <= n/m (seg_block=%d, n/m=%d)", B, L.nseg);
    P->B = B;
    P->grid = profile_grid(L.ntile * (int64_t)B, L.w);
    size_t o = 0;
    P->o_T = o;      o = al(o + L.sT.total);
    P->o_Dblk = o;   o = al(o + sizeof(float) * (size_t)B * L.Nm);
    P->o_P = o;      o = al(o + sizeof(float) * (size_t)K * L.Nm);
    P->o_M = o;      o = al(o + sizeof(float) * L.Nm);
    P->o_part = o;   o = al(o + sizeof(double) * (size_t)L.nseg * L.nblk);
    P->o_pick = o;   o = al(o + sizeof(int32_t) * K);
    P->o_area = o;   o = al(o + sizeof(double) * K);
    P->o_chosen = o; o = al(o + (size_t)L.nseg);
    P->o_count = o;  o = al(o + sizeof(int32_t) * K);
    P->o_iota = o;   o = al(o + sizeof(int32_t) * K);
    P->o_dmax = o;   o = al(o + 256);
    P->o_crit = o;   o = al(o + sizeof(double) * (L.nblk2 + 1));
    P->o_rw = o;     o = al(o + sizeof(float) * profile_scratch_bound(L.Nm, B, L.w));
    P->total = o;
    return PST_OK;
}

// Statistics of the rows of segments s0 .. : the series' own statistics
// shifted by s0 segments.
Stats rows_from(Stats s, int64_t off) {
    s.xc += off;
    s.mu += off;
    s.inv += off;
    s.h += off;
    s.df += off;
    s.dg += off;
    return s;
}

// With D_host (pinned, nseg x Nm floats) the profile set is computed once:
// round 0 copies every block out after its area partials, later rounds copy
// the blocks back instead of recomputing them, and the picked rows come from
// host memory too.  Without it every round recomputes the blocks.
int run_blocked(pst_ctx *c, const BlockedLayout &P, const double *T, char *ws, pst_snippet *out, float *profiles,
                int32_t *owner, float *dmax_host, double *score_host = nullptr, float *D_host = nullptr) {
    const Layout &L = P.L;
    int rc = series_stats(c, T, ws + P.o_T, L.sT, "T");
    if (rc) return rc;
    const Stats st = stats_view(ws + P.o_T, L.sT);
    unsigned *dmax = (unsigned *)(ws + P.o_dmax);
    HIPCHK(c, launch_fill_u32(dmax, 1, 0u, c->stream));
    std::vector<int32_t> iota(L.K);
    for (int p = 0; p < L.K; ++p) iota[p] = p;
    HIPCHK(c, hipMemcpyAsync(ws + P.o_iota, iota.data(), sizeof(int32_t) * L.K, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, profile_prepare(L.w));
    // greedy state for the whole set; D is only ever a block or the kept rows
    GreedyJob G{};
    G.ld = L.Nm;
    G.Nm = L.Nm;
    G.nseg = L.nseg;
    G.K = L.K;
    G.M = (float *)(ws + P.o_M);
    G.part = (double *)(ws + P.o_part);
    G.nblk = L.nblk;
    G.pick = (int32_t *)(ws + P.o_pick);
    G.area = (double *)(ws + P.o_area);
    G.chosen = (uint8_t *)(ws + P.o_chosen);
    G.count = (int32_t *)(ws + P.o_count);
    G.crit = nullptr;
    G.nblk2 = 0;
    float *Dblk = (float *)(ws + P.o_Dblk);
    float *Prow = (float *)(ws + P.o_P);
    HIPCHK(c, launch_greedy_init(G, c->stream));
    ProfileJob base = job_for(L, ws, Dblk, L.Nm, nullptr);
    base.col = st;
    base.rw = (float *)(ws + P.o_rw);
    base.anchor_every = c->opt_anchor;
    for (int r = 0; r < L.K; ++r) {
        for (int32_t s0 = 0; s0 < L.nseg; s0 += P.B) {
            const int32_t nb = std::min(P.B, L.nseg - s0);
            float *hblk = D_host ? D_host + (size_t)s0 * L.Nm : nullptr;
            if (r == 0 || !D_host) {
                ProfileJob j = base;
                j.row = rows_from(st, (int64_t)s0 * L.m);
                j.nq = nb;
                j.D = Dblk;
                j.dmax_bits = r == 0 ? dmax : nullptr;
                j.grid = profile_grid(L.ntile * (int64_t)nb, L.w);
                HIPCHK(c, launch_profile_batch(&j, 1, j.grid, nullptr, c->stream));
                if (D_host)
                    HIPCHK(c, hipMemcpyAsync(hblk, Dblk, sizeof(float) * (size_t)nb * L.Nm, hipMemcpyDeviceToHost,
                                             c->stream));
            } else {
                HIPCHK(c, hipMemcpyAsync(Dblk, hblk, sizeof(float) * (size_t)nb * L.Nm, hipMemcpyHostToDevice,
                                         c->stream));
            }
            GreedyJob Gb = G;
            Gb.D = Dblk;
            Gb.nseg = nb;
            Gb.part = G.part + (size_t)s0 * L.nblk;
            Gb.chosen = G.chosen + s0;
            HIPCHK(c, launch_area_parts(Gb, c->stream));
        }
        HIPCHK(c, launch_pick(G, r, c->stream));
        int32_t pk = 0;
        HIPCHK(c, hipMemcpyAsync(&pk, G.pick + r, sizeof pk, hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        // the picked segment's profile, kept as row r: recomputed alone, or
        // copied back from host memory
        if (D_host) {
            HIPCHK(c, hipMemcpyAsync(Prow + (size_t)r * L.Nm, D_host + (size_t)pk * L.Nm, sizeof(float) * L.Nm,
                                     hipMemcpyHostToDevice, c->stream));
        } else {
            ProfileJob j = base;
            j.row = rows_from(st, (int64_t)pk * L.m);
            j.nq = 1;
            j.D = Prow + (size_t)r * L.Nm;
            j.dmax_bits = nullptr;
            j.grid = profile_grid(L.ntile, L.w);
            HIPCHK(c, launch_profile_batch(&j, 1, j.grid, nullptr, c->stream));
        }
        GreedyJob Gk = G;
        Gk.D = Prow;
        Gk.pick = (int32_t *)(ws + P.o_iota);
        HIPCHK(c, launch_update_M(Gk, r, c->stream));
    }
    // neighbours and counts over the kept rows (row p = the p-th pick)
    GreedyJob Go = G;
    Go.D = Prow;
    Go.pick = (int32_t *)(ws + P.o_iota);
    Go.owner = owner;
    Go.profiles = profiles;
    HIPCHK(c, launch_owner(Go, c->stream));
    if (score_host) {  // eq. 18's numerator over the kept rows
        Go.crit = (double *)(ws + P.o_crit);
        Go.nblk2 = L.nblk2;
        HIPCHK(c, launch_criterion(Go, c->stream));
    }
    Layout Lr = L;  // collect_records reads picks, areas, counts, max and criterion at these offsets
    Lr.o_pick = P.o_pick;
    Lr.o_area = P.o_area;
    Lr.o_count = P.o_count;
    Lr.o_dmax = P.o_dmax;
    Lr.o_crit = P.o_crit;
    return collect_records(c, Lr, ws, out, dmax_host, score_host);
}

// ---------------------------------------------------------------- length sweep
// All candidate lengths of eq. 18 in one persistent profile launch, the greedy
// search / neighbours / criterion of each candidate after it, and a gather of
// the per-candidate scalars, optionally captured once as a HIP graph.

struct SweepPlan {
    int nm = 0, K = 0;
    int32_t wmax = 0, grid = 0;
    std::vector<int32_t> shape_w;  // widest w of each workgroup shape among the lengths, widest first
    std::vector<Layout> L;        // per candidate: sizes
    std::vector<int32_t> ls;      // distinct l
    std::vector<StatsLayout> SL;  // statistics layout per distinct l
    std::vector<size_t> o_stats;
    std::vector<int> li;          // candidate -> distinct-l index
    struct GB {
        size_t D, M, part, pick, area, chosen, count, crit, dmax;
    };
    std::vector<GB> gb;
    size_t o_rw = 0, o_counter = 0, o_out = 0, total = 0;
    int out_stride = 0;
};


// Lengths of each workgroup shape run in a launch of that shape: the widest
// w of every shape among the lengths, widest first (redone when a tuned
// geometry changes the shapes).
void sweep_shapes(SweepPlan *P) {
    P->grid = profile_slots(P->wmax);
    P->shape_w.clear();
    std::vector<int32_t> ws_sorted;
    for (const Layout &L : P->L) ws_sorted.push_back(L.w);
    std::sort(ws_sorted.begin(), ws_sorted.end(), std::greater<int32_t>());
    for (int32_t w : ws_sorted) {
        bool seen = false;
        for (int32_t v : P->shape_w) seen |= profile_shape(v) == profile_shape(w);
        if (!seen) P->shape_w.push_back(w);
    }
}

int plan_sweep(pst_ctx *c, int64_t n, const int32_t *m_list, int32_t nm, const int32_t *l_list,
               int32_t K, SweepPlan *P) {
    if (!m_list || nm < 1) return fail(c, PST_EINVAL, "empty candidate list");
    if (nm > kMaxJobs) return fail(c, PST_EINVAL, "at most %d candidate lengths per sweep", kMaxJobs);
    if (K < 1) return fail(c, PST_EINVAL, "need K >= 1 (K=%d)", K);
    P->nm = nm;
    P->K = K;
    P->L.resize(nm);
    P->li.resize(nm);
    P->gb.resize(nm);
    for (int i = 0; i < nm; ++i) {
        const int32_t l = l_list ? l_list[i] : m_list[i] / 2;
        const int rc = plan(c, n, m_list[i], l, 0, K, &P->L[i]);
        if (rc) return rc;
        P->wmax = std::max(P->wmax, P->L[i].w);
        int j = 0;
        while (j < (int)P->ls.size() && P->ls[j] != l) ++j;
        if (j == (int)P->ls.size()) P->ls.push_back(l);
        P->li[i] = j;
    }
    size_t o = 0;
    for (int32_t l : P->ls) {
        P->SL.push_back(stats_layout(n, l));
        P->o_stats.push_back(o);
        o = al(o + P->SL.back().total);
    }
    sweep_shapes(P);
    // scratch for any geometry of any length (one may be tuned after planning)
    size_t scratch = 0;
    for (int i = 0; i < nm; ++i)
        scratch = std::max(scratch, profile_scratch_bound(P->L[i].Nm, (int64_t)1 << 40, P->L[i].w));
    P->o_rw = o;
    o = al(o + sizeof(float) * scratch);
    P->o_counter = o;
    o = al(o + 256);
    for (int i = 0; i < nm; ++i) {
        const Layout &L = P->L[i];
        SweepPlan::GB &g = P->gb[i];
        g.D = o;      o = al(o + sizeof(float) * (size_t)L.nseg * L.Nm);
        g.M = o;      o = al(o + sizeof(float) * L.Nm);
        g.part = o;   o = al(o + sizeof(double) * (size_t)L.nseg * L.nblk);
        g.pick = o;   o = al(o + sizeof(int32_t) * K);
        g.area = o;   o = al(o + sizeof(double) * K);
        g.chosen = o; o = al(o + (size_t)L.nseg);
        g.count = o;  o = al(o + sizeof(int32_t) * K);
        g.crit = o;   o = al(o + sizeof(double) * (L.nblk2 + 1));
        g.dmax = o;   o = al(o + 256);
    }
    P->out_stride = 3 + 3 * K;
    P->o_out = o;
    o = al(o + sizeof(double) * nm * P->out_stride);
    P->total = o;
    return PST_OK;
}

GreedyJob sweep_greedy(const SweepPlan &P, int i, char *ws) {
    const Layout &L = P.L[i];
    const SweepPlan::GB &g = P.gb[i];
    GreedyJob G{};
    G.D = (const float *)(ws + g.D);
    G.ld = L.Nm;
    G.Nm = L.Nm;
    G.nseg = L.nseg;
    G.K = P.K;
    G.M = (float *)(ws + g.M);
    G.part = (double *)(ws + g.part);
    G.nblk = L.nblk;
    G.pick = (int32_t *)(ws + g.pick);
    G.area = (double *)(ws + g.area);
    G.chosen = (uint8_t *)(ws + g.chosen);
    G.count = (int32_t *)(ws + g.count);
    G.crit = (double *)(ws + g.crit);
    G.nblk2 = L.nblk2;
    return G;
}

int sweep_jobs(const SweepPlan &P, char *ws, int32_t grid, ProfileJob *jobs, int32_t anchor = 0) {
    std::vector<int> order(P.nm);
    for (int i = 0; i < P.nm; ++i) order[i] = i;
    // widest problems first: their tiles are the longest
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return P.L[a].w > P.L[b].w; });
    for (int j = 0; j < P.nm; ++j) {
        const int i = order[j];
        const Layout &L = P.L[i];
        ProfileJob J{};
        J.col = stats_view(ws + P.o_stats[P.li[i]], P.SL[P.li[i]]);
        J.row = J.col;
        J.row_stride = L.m;
        J.n = L.n;
        J.Nl = L.Nl;
        J.Nm = L.Nm;
        J.m = L.m;
        J.l = L.l;
        J.w = L.w;
        J.k = L.k;
        J.nq = L.nseg;
        J.D = (float *)(ws + P.gb[i].D);
        J.ld = L.Nm;
        J.rw = (float *)(ws + P.o_rw);
        J.dmax_bits = (unsigned *)(ws + P.gb[i].dmax);
        J.grid = grid;
        J.anchor_every = anchor;
        jobs[j] = J;
    }
    return P.nm;
}

// The profile launches of a sweep: one persistent launch per workgroup
// shape among the lengths, widest first, each grid scaled like the widest
// shape's (grid of P.grid).
hipError_t launch_sweep_profiles(const SweepPlan &P, char *ws, int32_t grid, bool dynamic, hipStream_t st,
                                 int32_t anchor, bool one_launch = false) {
    ProfileJob jobs[kMaxJobs];
    const int nj = sweep_jobs(P, ws, grid, jobs, anchor);
    uint32_t *counter = (uint32_t *)(ws + P.o_counter);
    hipError_t e;
    if (one_launch) {  // every length in the widest one's geometry
        if ((e = launch_fill_u32(counter, 1, 0u, st)) != hipSuccess) return e;
        return launch_profile_batch(jobs, nj, grid, dynamic ? counter : nullptr, st);
    }
    int done = 0;
    for (int32_t wg : P.shape_w) {
        const int32_t shape = profile_shape(wg);
        std::stable_partition(jobs + done, jobs + nj, [&](const ProfileJob &j) { return profile_shape(j.w) == shape; });
        int cnt = 0;
        while (done + cnt < nj && profile_shape(jobs[done + cnt].w) == shape) ++cnt;
        if (cnt == 0) continue;
        const int32_t g = std::max<int32_t>(1, (int32_t)((int64_t)profile_slots(wg) * grid / P.grid));
        for (int j = done; j < done + cnt; ++j) jobs[j].grid = g;
        if ((e = launch_fill_u32(counter, 1, 0u, st)) != hipSuccess) return e;
        if ((e = launch_profile_batch(jobs + done, cnt, g, dynamic ? counter : nullptr, st)) != hipSuccess) return e;
        done += cnt;
    }
    return hipSuccess;
}

hipError_t enqueue_sweep(const SweepPlan &P, const double *T, char *ws, int32_t grid, bool dynamic,
                         hipStream_t st, int32_t anchor, bool one_launch) {
    hipError_t e;
    for (size_t j = 0; j < P.ls.size(); ++j)
        if ((e = launch_series_stats(T, ws + P.o_stats[j], P.SL[j], st)) != hipSuccess) return e;
    for (int i = 0; i < P.nm; ++i)
        if ((e = launch_fill_u32((uint32_t *)(ws + P.gb[i].dmax), 1, 0u, st)) != hipSuccess) return e;
    if ((e = launch_sweep_profiles(P, ws, grid, dynamic, st, anchor, one_launch)) != hipSuccess) return e;
    SweepGather Gt{};
    Gt.nm = P.nm;
    Gt.K = P.K;
    Gt.out = (double *)(ws + P.o_out);
    // every length's greedy search and neighbours in the same launches
    GreedyJob gs[kMaxJobs];
    for (int i = 0; i < P.nm; ++i) gs[i] = sweep_greedy(P, i, ws);
    if ((e = launch_greedy_batch(gs, P.nm, st)) != hipSuccess) return e;
    if ((e = launch_owner_batch(gs, P.nm, st)) != hipSuccess) return e;
    for (int i = 0; i < P.nm; ++i) {
        const GreedyJob &G = gs[i];
        if ((e = launch_criterion(G, st)) != hipSuccess) return e;
        Gt.crit[i] = G.crit + G.nblk2;
        Gt.dmax[i] = (const uint32_t *)(ws + P.gb[i].dmax);
        Gt.bad[i] = stats_misc(ws + P.o_stats[P.li[i]], P.SL[P.li[i]]) + 2;
        Gt.area[i] = G.area;
        Gt.pick[i] = G.pick;
        Gt.count[i] = G.count;
    }
    return launch_gather(Gt, st);
}

// ---- autotuner: persistent grid size and tile scheduling of the batched
// profile launch, timed on the caller's own problem the first time a shape
// bucket is seen; remembered per process and optionally in a text file named
// by PST_AUTOTUNE_CACHE ("arch wmax tiles_log2 grid dynamic ms" per line).
// The choice only moves tiles between workgroups: results are identical.
using TuneKey = std::tuple<std::string, int, int>;
struct TuneVal {
    int grid, dynamic;
    float ms;
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneVal> g_tuned;
bool g_tune_loaded = false;

// Tile geometries chosen per (arch, w), from timing or the cache file.
std::map<std::pair<std::string, int>, std::pair<int32_t, float>> g_geo_tuned;

void tune_load_locked() {
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *path = std::getenv("PST_AUTOTUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char line[256];
    while (std::fgets(line, sizeof line, f)) {
        char arch[64];
        int wm, tl, gr, dy, code;
        float ms;
        if (std::sscanf(line, "geo %63s %d %d %f", arch, &wm, &code, &ms) == 4)
            g_geo_tuned[{arch, wm}] = {code, ms};
        else if (std::sscanf(line, "%63s %d %d %d %d %f", arch, &wm, &tl, &gr, &dy, &ms) == 6)
            g_tuned[TuneKey(arch, wm, tl)] = TuneVal{gr, dy, ms};
    }
    std::fclose(f);
}

std::string device_arch(pst_ctx *c) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c->device) != hipSuccess) return "unknown";
    return std::string(prop.gcnArchName).substr(0, 6);
}

// The tile geometry of one profile job's w: every candidate the kernels can
// run is timed on the same queries of the job (as many as give about sixteen
// tiles per resident workgroup of the geometry in use: long enough to measure,
// short enough to repeat; best of three launches after a warm-up), the
// fastest is installed for that w process-wide and
// appended to the cache file; a w seen before (in this process or the file)
// takes the remembered choice without timing.  The job's statistics must be
// in place; its D rows are overwritten.
int tune_geometry_job(pst_ctx *c, ProfileJob J, int32_t *code_out, float *ms_out) {
    const std::string arch = device_arch(c);
    const int32_t w = J.w;
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        tune_load_locked();
        auto it = g_geo_tuned.find({arch, w});
        if (it != g_geo_tuned.end() && profile_set_geometry(w, it->second.first)) {
            *code_out = it->second.first;
            *ms_out = it->second.second;
            return PST_OK;
        }
    }
    int32_t codes[64];
    const int nc = std::min<int>(profile_geometry_candidates(w, codes, 64), 64);
    hipEvent_t a, b;
    HIPCHK(c, hipEventCreate(&a));
    HIPCHK(c, hipEventCreate(&b));
    int32_t best = profile_geometry(w);
    float best_ms = 1e30f;
    // the same queries for every candidate: enough for about sixteen tiles
    // per resident workgroup of the geometry in use
    const int64_t tq0 = (J.Nm + profile_tile_windows(w) - 1) / profile_tile_windows(w);
    const int32_t nq = (int32_t)std::max<int64_t>(
        1, std::min<int64_t>(J.nq, (16 * (int64_t)profile_slots(w) + tq0 - 1) / tq0));
    for (int i = 0; i < nc; ++i) {
        if (!profile_set_geometry(w, codes[i])) continue;
        ProfileJob j = J;
        const int64_t tiles_per_q = (j.Nm + profile_tile_windows(w) - 1) / profile_tile_windows(w);
        j.nq = nq;
        j.grid = profile_grid(tiles_per_q * j.nq, w);
        float ms = 1e30f;
        hipError_t e = profile_prepare(w);
        for (int rep = 0; rep < 4 && e == hipSuccess; ++rep) {  // a warm-up, then the best of three
            if ((e = hipEventRecord(a, c->stream)) != hipSuccess) break;
            if ((e = launch_profile_batch(&j, 1, j.grid, nullptr, c->stream)) != hipSuccess) break;
            if ((e = hipEventRecord(b, c->stream)) != hipSuccess) break;
            if ((e = hipEventSynchronize(b)) != hipSuccess) break;
            float t = 0.0f;
            if ((e = hipEventElapsedTime(&t, a, b)) != hipSuccess) break;
            if (rep > 0) ms = std::min(ms, t);
        }
        if (e != hipSuccess) {
            (void)profile_set_geometry(w, 0);
            (void)hipEventDestroy(a);
            (void)hipEventDestroy(b);
            return fail(c, PST_EDEVICE, "geometry tuning launch failed: %s", hipGetErrorString(e));
        }
        if (ms < best_ms) {
            best_ms = ms;
            best = codes[i];
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)profile_set_geometry(w, best);
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_geo_tuned[{arch, w}] = {best, best_ms};
    if (const char *path = std::getenv("PST_AUTOTUNE_CACHE")) {
        if (FILE *f = std::fopen(path, "a")) {
            std::fprintf(f, "geo %s %d %d %.4f\n", arch.c_str(), w, best, best_ms);
            std::fclose(f);
        }
    }
    *code_out = best;
    *ms_out = best_ms;
    return PST_OK;
}

int64_t sweep_tiles(const SweepPlan &P) {
    const int JT = profile_tile_windows(P.wmax);
    int64_t t = 0;
    for (const Layout &L : P.L) t += ((L.Nm + JT - 1) / JT) * (int64_t)L.nseg;
    return t;
}

int autotune(pst_ctx *c, const SweepPlan &P, const double *T, char *ws, TuneVal *out) {
    hipDeviceProp_t prop;
    HIPCHK(c, hipGetDeviceProperties(&prop, c->device));
    const int64_t tiles = sweep_tiles(P);
    const int tl = tiles > 1 ? (int)std::floor(std::log2((double)tiles)) : 0;
    const TuneKey key(std::string(prop.gcnArchName).substr(0, 6), P.wmax, tl);
    {
        std::lock_guard<std::mutex> g(g_tune_mu);
        tune_load_locked();
        auto it = g_tuned.find(key);
        if (it != g_tuned.end()) {
            // a line of the cache file may come from another build: never more
            // workgroups than the workspace has scratch slots for
            *out = it->second;
            out->grid = std::max(1, std::min(out->grid, P.grid));
            out->dynamic = out->dynamic != 0;
            return PST_OK;
        }
    }
    // statistics once, then each candidate configuration of the profile launch
    for (size_t j = 0; j < P.ls.size(); ++j)
        HIPCHK(c, launch_series_stats(T, ws + P.o_stats[j], P.SL[j], c->stream));
    // grid: all resident workgroups, three quarters, half; tiles striped or
    // handed out by the device counter
    const int S = P.grid;
    const int cand[][2] = {{S, 1}, {S, 0}, {S * 3 / 4, 1}, {S / 2, 1}};
    hipEvent_t a, b;
    HIPCHK(c, hipEventCreate(&a));
    HIPCHK(c, hipEventCreate(&b));
    TuneVal best{S, 1, 1e30f};
    for (int32_t wg : P.shape_w) HIPCHK(c, profile_prepare(wg));
    for (const auto &cf : cand) {
        HIPCHK(c, hipEventRecord(a, c->stream));
        HIPCHK(c, launch_sweep_profiles(P, ws, cf[0], cf[1] != 0, c->stream, 0));
        HIPCHK(c, hipEventRecord(b, c->stream));
        HIPCHK(c, hipEventSynchronize(b));
        float ms = 0.0f;
        HIPCHK(c, hipEventElapsedTime(&ms, a, b));
        if (ms < best.ms) best = TuneVal{cf[0], cf[1], ms};
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tuned[key] = best;
    if (const char *path = std::getenv("PST_AUTOTUNE_CACHE")) {
        if (FILE *f = std::fopen(path, "a")) {
            std::fprintf(f, "%s %d %d %d %d %.4f\n", std::get<0>(key).c_str(), P.wmax, tl, best.grid,
                         best.dynamic, best.ms);
            std::fclose(f);
        }
    }
    *out = best;
    return PST_OK;
}

int run_sweep(pst_ctx *c, const SweepPlan &P, const double *T, char *ws, size_t ws_bytes,
              const int32_t *m_list, const int32_t *l_list, std::vector<double> *res) {
    TuneVal cfg{c->opt_grid > 0 ? std::min(c->opt_grid, P.grid) : P.grid, c->opt_dynamic, 0.0f};
    if (c->opt_autotune) {
        const int rc = autotune(c, P, T, ws, &cfg);
        if (rc) return rc;
    }
    for (int32_t wg : P.shape_w) HIPCHK(c, profile_prepare(wg));
    if (!c->opt_graph) {
        HIPCHK(c, enqueue_sweep(P, T, ws, cfg.grid, cfg.dynamic != 0, c->stream, c->opt_anchor, c->opt_one_launch));
    } else {
        std::vector<int64_t> key = {(int64_t)(uintptr_t)T, P.L[0].n, (int64_t)(uintptr_t)ws,
                                    (int64_t)ws_bytes, P.nm, P.K, cfg.grid, cfg.dynamic, c->opt_anchor,
                                    c->opt_one_launch};
        for (int i = 0; i < P.nm; ++i) {
            key.push_back(m_list[i]);
            key.push_back(l_list ? l_list[i] : m_list[i] / 2);
            key.push_back(profile_geometry(P.L[i].w));
        }
        hipGraphExec_t exec = nullptr;
        for (const GraphEntry &g : c->graphs)
            if (g.key == key) exec = g.exec;
        if (!exec) {
            if (!c->cap) HIPCHK(c, hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking));
            HIPCHK(c, hipStreamBeginCapture(c->cap, hipStreamCaptureModeRelaxed));
            const hipError_t eq =
                enqueue_sweep(P, T, ws, cfg.grid, cfg.dynamic != 0, c->cap, c->opt_anchor, c->opt_one_launch);
            hipGraph_t graph = nullptr;
            const hipError_t ee = hipStreamEndCapture(c->cap, &graph);
            HIPCHK(c, eq);
            HIPCHK(c, ee);
            const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            HIPCHK(c, ei);
            c->graphs.push_back(GraphEntry{key, exec});
        }
        HIPCHK(c, hipGraphLaunch(exec, c->stream));
    }
    res->assign((size_t)P.nm * P.out_stride, 0.0);
    HIPCHK(c, hipMemcpyAsync(res->data(), ws + P.o_out, sizeof(double) * res->size(),
                             hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PST_OK;
}

}  // namespace

extern "C" {

const char *pst_version(void) { return "pst 0.1 (gfx950)"; }

int pst_create(pst_ctx **out, int device, void *hip_stream) {
    if (!out) return PST_EINVAL;
    *out = nullptr;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return PST_EDEVICE;
    pst_ctx *c = new pst_ctx;
    c->device = device;
    c->stream = (hipStream_t)hip_stream;
    c->poisoned = false;
    c->timing = false;
    c->timed = false;
    c->ev0 = c->ev1 = nullptr;
    c->cap = nullptr;
    c->err[0] = 0;
    // the device address of the fixed scratch of pst_mpdist_profile_noalloc,
    // looked up once per device with that device current
    c->fixed_scratch = nullptr;
    int prev = -1;
    if (hipGetDevice(&prev) == hipSuccess && hipSetDevice(device) == hipSuccess) {
        if (static_scratch(device, &c->fixed_scratch) != hipSuccess) c->fixed_scratch = nullptr;
        (void)hipSetDevice(prev);
    }
    (void)hipGetLastError();
    *out = c;
    return PST_OK;
}

void pst_destroy(pst_ctx *ctx) {
    if (!ctx) return;
    for (GraphEntry &g : ctx->graphs) (void)hipGraphExecDestroy(g.exec);
    if (ctx->cap) (void)hipStreamDestroy(ctx->cap);
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    delete ctx;
}

int pst_set_timing(pst_ctx *ctx, int on) {
    int rc = begin(ctx);
    if (rc) return rc;
    if (on && !ctx->ev0) {
        HIPCHK(ctx, hipEventCreate(&ctx->ev0));
        HIPCHK(ctx, hipEventCreate(&ctx->ev1));
    }
    ctx->timing = on != 0;
    ctx->timed = false;
    return PST_OK;
}

int pst_last_profile_ms(pst_ctx *ctx, float *ms) {
    int rc = begin(ctx);
    if (rc) return rc;
    if (!ms) return fail(ctx, PST_EINVAL, "ms is NULL");
    if (!ctx->timed) return fail(ctx, PST_ENOTREADY, "no timed call");
    HIPCHK(ctx, hipEventSynchronize(ctx->ev1));
    HIPCHK(ctx, hipEventElapsedTime(ms, ctx->ev0, ctx->ev1));
    return PST_OK;
}

const char *pst_last_error(const pst_ctx *ctx) { return ctx ? ctx->err : "null context"; }

size_t pst_workspace_bytes(int64_t n, int32_t m, int32_t l, int32_t K) {
    Layout L;
    if (plan(nullptr, n, m, l, 0, K, &L) != PST_OK) return 0;
    return L.total;
}

size_t pst_select_length_workspace_bytes(int64_t n, const int32_t *m_list, int32_t num_m,
                                         const int32_t *l_list, int32_t K) {
    SweepPlan P;
    if (plan_sweep(nullptr, n, m_list, num_m, l_list, K, &P) != PST_OK) return 0;
    size_t mx = P.total;  // the per-length path needs at most the largest single layout
    for (const Layout &L : P.L) mx = std::max(mx, L.total);
    return mx;
}

namespace {
// Workspace of the labelling score: confusion counts, then the results.
struct LabelLayout {
    size_t conf, bad, map, prec, rec, f1, macro, total;
};
bool label_layout(int32_t K, int32_t C, LabelLayout *L) {
    if (K < 1 || C < 1 || K > (1 << 20) || C > 4096 || (int64_t)K * C > (1 << 26)) return false;
    size_t o = 0;
    L->conf = o;  o = al(o + sizeof(unsigned) * (size_t)K * C);
    L->bad = o;   o = al(o + sizeof(unsigned));
    L->map = o;   o = al(o + sizeof(int32_t) * K);
    L->prec = o;  o = al(o + sizeof(double) * C);
    L->rec = o;   o = al(o + sizeof(double) * C);
    L->f1 = o;    o = al(o + sizeof(double) * C);
    L->macro = o; o = al(o + sizeof(double));
    L->total = o;
    return true;
}
}  // namespace

size_t pst_label_workspace_bytes(int32_t K, int32_t C) {
    LabelLayout L;
    return label_layout(K, C, &L) ? L.total : 0;
}

int pst_label_f1(pst_ctx *ctx, const int32_t *owner_dev, int64_t n, int32_t m, int32_t K,
                 const int32_t *truth_dev, int32_t C, int32_t *map_host, double *precision_host,
                 double *recall_host, double *f1_host, double *macro_f1_host, void *ws_dev, size_t ws_bytes) {
    int rc = begin(ctx);
    if (rc) return rc;
    LabelLayout LL;
    if (!label_layout(K, C, &LL)) return fail(ctx, PST_EINVAL, "bad K=%d or C=%d", K, C);
    if (m < 1 || n < m) return fail(ctx, PST_EINVAL, "need 1 <= m <= n (n=%lld m=%d)", (long long)n, m);
    if (!owner_dev || !truth_dev || !macro_f1_host) return fail(ctx, PST_EINVAL, "null pointer argument");
    if (!ws_dev) return fail(ctx, PST_EINVAL, "workspace is NULL");
    if (((uintptr_t)ws_dev & 255) != 0) return fail(ctx, PST_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < LL.total) return fail(ctx, PST_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, LL.total);
    char *ws = (char *)ws_dev;
    LabelJob J;
    J.owner = owner_dev;
    J.truth = truth_dev;
    J.n = n;
    J.m = m;
    J.K = K;
    J.C = C;
    J.lds = false;
    J.conf = (unsigned *)(ws + LL.conf);
    J.bad = (unsigned *)(ws + LL.bad);
    J.map = (int32_t *)(ws + LL.map);
    J.prec = (double *)(ws + LL.prec);
    J.rec = (double *)(ws + LL.rec);
    J.f1 = (double *)(ws + LL.f1);
    J.macro = (double *)(ws + LL.macro);
    HIPCHK(ctx, launch_label_f1(J, ctx->stream));
    unsigned bad = 0;
    HIPCHK(ctx, hipMemcpyAsync(&bad, J.bad, sizeof bad, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(macro_f1_host, J.macro, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    if (map_host)
        HIPCHK(ctx, hipMemcpyAsync(map_host, J.map, sizeof(int32_t) * K, hipMemcpyDeviceToHost, ctx->stream));
    if (precision_host)
        HIPCHK(ctx, hipMemcpyAsync(precision_host, J.prec, sizeof(double) * C, hipMemcpyDeviceToHost, ctx->stream));
    if (recall_host)
        HIPCHK(ctx, hipMemcpyAsync(recall_host, J.rec, sizeof(double) * C, hipMemcpyDeviceToHost, ctx->stream));
    if (f1_host)
        HIPCHK(ctx, hipMemcpyAsync(f1_host, J.f1, sizeof(double) * C, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (bad) return fail(ctx, PST_EINVAL, "%u elements have an owner outside [0, K) or a class outside [0, C)", bad);
    return PST_OK;
}

int pst_tune_geometry(pst_ctx *ctx, const double *T_dev, int64_t n, int32_t m, int32_t l, int32_t *code_out,
                      float *ms_out, void *ws_dev, size_t ws_bytes) {
    int rc = begin(ctx);
    if (rc) return rc;
    Layout L;
    if ((rc = plan(ctx, n, m, l, 0, 1, &L))) return rc;
    if (!T_dev || !code_out) return fail(ctx, PST_EINVAL, "null pointer argument");
    if ((rc = check_ws(ctx, L, ws_dev, ws_bytes))) return rc;
    char *ws = (char *)ws_dev;
    if ((rc = series_stats(ctx, T_dev, ws + L.o_T, L.sT, "T"))) return rc;
    float ms = 0.0f;
    if ((rc = tune_geometry_job(ctx, job_for(L, ws, (float *)(ws + L.o_D), L.Nm, nullptr), code_out, &ms)))
        return rc;
    if (ms_out) *ms_out = ms;
    return PST_OK;
}

int pst_geometry_candidates(int32_t w, int32_t *codes, int32_t max) {
    if (max < 0 || (max > 0 && !codes)) return PST_EINVAL;
    return profile_geometry_candidates(w, codes, max);
}

int32_t pst_geometry(int32_t w) { return w >= 1 && w <= kMaxW ? profile_geometry(w) : 0; }

int pst_set_geometry(int32_t w, int32_t code) { return profile_set_geometry(w, code) ? PST_OK : PST_EINVAL; }

int pst_set_option(pst_ctx *ctx, int option, int64_t value) {
    if (!ctx) return PST_EINVAL;
    switch (option) {
        case PST_OPT_SWEEP_GRAPH: ctx->opt_graph = value != 0; break;
        case PST_OPT_AUTOTUNE: ctx->opt_autotune = value != 0; break;
        case PST_OPT_TUNE_GEOMETRY: ctx->opt_tune_geometry = value != 0; break;
        case PST_OPT_SWEEP_ONE_LAUNCH: ctx->opt_one_launch = value != 0; break;
        case PST_OPT_PROFILE_GRID:
            if (value < 0 || value > 4096) return fail(ctx, PST_EINVAL, "grid out of range");
            ctx->opt_grid = (int)value;
            break;
        case PST_OPT_DYNAMIC_TILES: ctx->opt_dynamic = value != 0; break;
        case PST_OPT_SWEEP_BATCHED: ctx->opt_batched = value != 0; break;
        case PST_OPT_ANCHOR_EVERY:
            if (value < 0 || value > (1 << 30)) return fail(ctx, PST_EINVAL, "anchor interval out of range");
            ctx->opt_anchor = (int)value;
            break;
        default: return fail(ctx, PST_EINVAL, "unknown option %d", option);
    }
    return PST_OK;
}

int pst_mpdist_profile(pst_ctx *ctx, const double *T_dev, int64_t n, const double *Q_dev, int32_t m,
                       int32_t l, int32_t k, float *out_dev, void *ws_dev, size_t ws_bytes) {
    int rc = begin(ctx);
    if (rc) return rc;
    Layout L;
    if ((rc = plan(ctx, n, m, l, k, 0, &L))) return rc;
    if (!T_dev || !Q_dev || !out_dev) return fail(ctx, PST_EINVAL, "null pointer argument");
    if ((rc = check_ws(ctx, L, ws_dev, ws_bytes))) return rc;
    char *ws = (char *)ws_dev;
    if ((rc = series_stats(ctx, T_dev, ws + L.o_T, L.sT, "T"))) return rc;
    if ((rc = series_stats(ctx, Q_dev, ws + L.o_Q, L.sQ, "Q"))) return rc;
    ProfileJob j = job_for(L, ws, out_dev, L.Nm, nullptr);
    j.row = stats_view(ws + L.o_Q, L.sQ);
    j.row_stride = 0;
    j.nq = 1;
    j.grid = profile_grid(L.ntile, L.w);
    HIPCHK(ctx, timed_profile(ctx, j));
    return PST_OK;
}

int pst_mpdist_profile_noalloc(pst_ctx *ctx, const double *T_dev, int64_t n, const double *Q_dev, int32_t m,
                               int32_t l, int32_t k, float *out_dev) {
    int rc = begin(ctx);
    if (rc) return rc;
    Layout L;
    if ((rc = plan(ctx, n, m, l, k, 0, &L, false))) return rc;
    if (!T_dev || !Q_dev || !out_dev) return fail(ctx, PST_EINVAL, "null pointer argument");
    if (!ctx->fixed_scratch) return fail(ctx, PST_EDEVICE, "the fixed device scratch is not available");
    // the statistics of T and Q (at the head of the workspace layout), then
    // profile scratch for as many persistent workgroups as fit (at least one)
    const size_t cap = static_scratch_bytes();
    const size_t used = al(L.o_Q + L.sQ.total);
    const size_t slot = sizeof(float) * profile_scratch_floats(1, L.w);
    if (used + slot > cap)
        return fail(ctx, PST_EINVAL, "n=%lld, m=%d, l=%d needs %zu bytes of scratch, the fixed scratch holds %zu",
                    (long long)n, m, l, used + slot, cap);
    char *ws = (char *)ctx->fixed_scratch;
    if ((rc = series_stats(ctx, T_dev, ws + L.o_T, L.sT, "T"))) return rc;
    if ((rc = series_stats(ctx, Q_dev, ws + L.o_Q, L.sQ, "Q"))) return rc;
    ProfileJob j = job_for(L, ws, out_dev, L.Nm, nullptr);
    j.row = stats_view(ws + L.o_Q, L.sQ);
    j.row_stride = 0;
    j.nq = 1;
    j.rw = (float *)(ws + used);
    j.grid = (int32_t)std::min<int64_t>(profile_grid(L.ntile, L.w), (int64_t)((cap - used) / slot));
    HIPCHK(ctx, timed_profile(ctx, j));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return PST_OK;
}

int pst_profile_set(pst_ctx *ctx, const double *T_dev, int64_t n, int32_t m, int32_t l, int32_t k,
                    float *D_dev, int64_t ld, float *dmax_dev, void *ws_dev, size_t ws_bytes) {
    int rc = begin(ctx);
    if (rc) return rc;
    Layout L;
    if ((rc = plan(ctx, n, m, l, k, 0, &L))) return rc;
    if (!T_dev || !D_dev) return fail(ctx, PST_EINVAL, "null pointer argument");
    if (ld < L.Nm) return fail(ctx, PST_EINVAL, "ld (%lld) < n-m+1 (%lld)", (long long)ld, (long long)L.Nm);
    if ((rc = check_ws(ctx, L, ws_dev, ws_bytes))) return rc;
    char *ws = (char *)ws_dev;
    if ((rc = series_stats(ctx, T_dev, ws + L.o_T, L.sT, "T"))) return rc;
    unsigned *dmax = (unsigned *)(ws + L.o_dmax);
    HIPCHK(ctx, launch_fill_u32(dmax, 1, 0u, ctx->stream));
    HIPCHK(ctx, timed_profile(ctx, job_for(L, ws, D_dev, ld, dmax)));
    if (dmax_dev)
        HIPCHK(ctx, hipMemcpyAsync(dmax_dev, dmax, sizeof(float), hipMemcpyDeviceToDevice, ctx->stream));
    return PST_OK;
}

int pst_snippets(pst_ctx *ctx, const double *T_dev, int64_t n, int32_t m, int32_t l, int32_t k,
                 int32_t K, pst_snippet *out_host, float *profiles_dev, int32_t *owner_dev,
                 float *dmax_host, void *ws_dev, size_t ws_bytes) {
    int rc = begin(ctx);
    if (rc) return rc;
    if (K < 1) return fail(ctx, PST_EINVAL, "need K >= 1 (K=%d)", K);
    Layout L;
    if ((rc = plan(ctx, n, m, l, k, K, &L))) return rc;
    if (!T_dev || !out_host) return fail(ctx, PST_EINVAL, "null pointer argument");
    if ((rc = check_ws(ctx, L, ws_dev, ws_bytes))) return rc;
    char *ws = (char *)ws_dev;
    if ((rc = snippets_device(ctx, T_dev, L, ws, owner_dev, profiles_dev, false))) return rc;
    return collect_records(ctx, L, ws, out_host, dmax_host, nullptr);
}

size_t pst_snippets_blocked_workspace_bytes(int64_t n, int32_t m, int32_t l, int32_t K, int32_t seg_block) {
    BlockedLayout P;
    if (plan_blocked(nullptr, n, m, l, 0, K, seg_block, &P) != PST_OK) return 0;
    return P.total;
}

int32_t pst_snippets_blocked_max_block(int64_t n, int32_t m, int32_t l, int32_t K, size_t budget_bytes) {
    Layout L;
    if (K < 1 || plan(nullptr, n, m, l, 0, K, &L, false) != PST_OK) return 0;
    // the workspace grows with the block: largest block that fits, by bisection
    int32_t lo = 0, hi = L.nseg;
    while (lo < hi) {
        const int32_t mid = lo + (hi - lo + 1) / 2;
        if (pst_snippets_blocked_workspace_bytes(n, m, l, K, mid) <= budget_bytes) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

int pst_snippets_blocked(pst_ctx *ctx, const double *T_dev, int64_t n, int32_t m, int32_t l, int32_t k, int32_t K,
                         int32_t seg_block, pst_snippet *out_host, float *profiles_dev, int32_t *owner_dev,
                         float *dmax_host, void *ws_dev, size_t ws_bytes) {
    int rc = begin(ctx);
    if (rc) return rc;
    BlockedLayout P;
    if ((rc = plan_blocked(ctx, n, m, l, k, K, seg_block, &P))) return rc;
    if (!T_dev || !out_host) return fail(ctx, PST_EINVAL, "null pointer argument");
    if (!ws_dev) return fail(ctx, PST_EINVAL, "workspace is NULL");
    if (((uintptr_t)ws_dev & 255) != 0) return fail(ctx, PST_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < P.total) return fail(ctx, PST_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, P.total);
    return run_blocked(ctx, P, T_dev, (char *)ws_dev, out_host, profiles_dev, owner_dev, dmax_host);
}

int pst_snippets_spilled(pst_ctx *ctx, const double *T_dev, int64_t n, int32_t m, int32_t l, int32_t k, int32_t K,
                         int32_t seg_block, float *D_host, pst_snippet *out_host, float *profiles_dev,
                         int32_t *owner_dev, float *dmax_host, void *ws_dev, size_t ws_bytes) {
    int rc = begin(ctx);
    if (rc) return rc;
    BlockedLayout P;
    if ((rc = plan_blocked(ctx, n, m, l, k, K, seg_block, &P))) return rc;
    if (!T_dev || !out_host || !D_host) return fail(ctx, PST_EINVAL, "null pointer argument");
    if (!ws_dev) return fail(ctx, PST_EINVAL, "workspace is NULL");
    if (((uintptr_t)ws_dev & 255) != 0) return fail(ctx, PST_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < P.total) return fail(ctx, PST_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, P.total);
    return run_blocked(ctx, P, T_dev, (char *)ws_dev, out_host, profiles_dev, owner_dev, dmax_host, nullptr, D_host);
}

size_t pst_select_length_blocked_workspace_bytes(int64_t n, const int32_t *m_list, int32_t num_m,
                                                 const int32_t *l_list, int32_t K, int32_t seg_block) {
    if (!m_list || num_m < 1 || num_m > kMaxJobs || seg_block < 1) return 0;
    size_t mx = 0;
    for (int i = 0; i < num_m; ++i) {
        const int32_t l = l_list ? l_list[i] : m_list[i] / 2;
        if (m_list[i] < 1) return 0;
        const int64_t nseg = n / m_list[i];
        const size_t b = pst_snippets_blocked_workspace_bytes(n, m_list[i], l, K, (int32_t)std::min<int64_t>(seg_block, nseg));
        if (b == 0) return 0;
        mx = std::max(mx, b);
    }
    return mx;
}

int pst_select_length_blocked(pst_ctx *ctx, const double *T_dev, int64_t n, const int32_t *m_list, int32_t num_m,
                              const int32_t *l_list, int32_t K, int32_t seg_block, int32_t *m_best,
                              double *scores_host, pst_snippet *out_host, float *profiles_dev, int32_t *owner_dev,
                              void *ws_dev, size_t ws_bytes) {
    int rc = begin(ctx);
    if (rc) return rc;
    if (!m_list || num_m < 1 || !m_best || !T_dev)
        return fail(ctx, PST_EINVAL, "need a candidate list, m_best and T");
    if (num_m > kMaxJobs) return fail(ctx, PST_EINVAL, "at most %d candidate lengths", kMaxJobs);
    if (seg_block < 1) return fail(ctx, PST_EINVAL, "need seg_block >= 1 (seg_block=%d)", seg_block);
    if (!ws_dev) return fail(ctx, PST_EINVAL, "workspace is NULL");
    if (((uintptr_t)ws_dev & 255) != 0) return fail(ctx, PST_EINVAL, "workspace must be 256-byte aligned");
    std::vector<BlockedLayout> P(num_m);
    for (int i = 0; i < num_m; ++i) {
        const int32_t l = l_list ? l_list[i] : m_list[i] / 2;
        if (m_list[i] < 2) return fail(ctx, PST_EINVAL, "need m >= 2 (m=%d)", m_list[i]);
        const int32_t B = (int32_t)std::min<int64_t>(seg_block, n / m_list[i]);
        if ((rc = plan_blocked(ctx, n, m_list[i], l, 0, K, std::max(B, 1), &P[i]))) return rc;
        if (ws_bytes < P[i].total)
            return fail(ctx, PST_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, P[i].total);
    }
    char *ws = (char *)ws_dev;
    int best = -1;
    double best_score = 0.0;
    for (int i = 0; i < num_m; ++i) {
        double score = 0.0;
        if ((rc = run_blocked(ctx, P[i], T_dev, ws, nullptr, nullptr, nullptr, nullptr, &score))) return rc;
        if (scores_host) scores_host[i] = score;
        if (best < 0 || score > best_score || (score == best_score && m_list[i] < m_list[best])) {
            best = i;
            best_score = score;
        }
    }
    *m_best = m_list[best];
    // the chosen length once more, now keeping its snippets, owners and profiles
    return run_blocked(ctx, P[best], T_dev, ws, out_host, profiles_dev, owner_dev, nullptr);
}

size_t pst_snippets_multi_workspace_bytes(int32_t d, int64_t n, int32_t m, int32_t l, int32_t K) {
    MultiPlan P;
    if (plan_multi(nullptr, d, n, m, l, 0, K, &P) != PST_OK) return 0;
    return P.total;
}

int pst_snippets_multi(pst_ctx *ctx, const double *T_dev, int32_t d, int64_t ld, int64_t n, int32_t m,
                       int32_t l, int32_t k, int32_t K, pst_snippet *out_host, int32_t *owner_dev,
                       float *dmax_host, void *ws_dev, size_t ws_bytes) {
    int rc = begin(ctx);
    if (rc) return rc;
    MultiPlan P;
    if ((rc = plan_multi(ctx, d, n, m, l, k, K, &P))) return rc;
    if (!T_dev || !out_host) return fail(ctx, PST_EINVAL, "null pointer argument");
    if (ld < n) return fail(ctx, PST_EINVAL, "ld (%lld) < n (%lld)", (long long)ld, (long long)n);
    if (!ws_dev) return fail(ctx, PST_EINVAL, "workspace is NULL");
    if (((uintptr_t)ws_dev & 255) != 0) return fail(ctx, PST_EINVAL, "workspace must be 256-byte aligned");
    if (ws_bytes < P.total) return fail(ctx, PST_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, P.total);
    return run_multi(ctx, P, T_dev, ld, (char *)ws_dev, out_host, owner_dev, dmax_host);
}

int pst_select_length(pst_ctx *ctx, const double *T_dev, int64_t n, const int32_t *m_list,
                      int32_t num_m, const int32_t *l_list, int32_t K, int32_t *m_best,
                      double *scores_host, pst_snippet *out_host, float *profiles_dev,
                      int32_t *owner_dev, void *ws_dev, size_t ws_bytes) {
    int rc = begin(ctx);
    if (rc) return rc;
    if (!m_list || num_m < 1 || !m_best || !T_dev)
        return fail(ctx, PST_EINVAL, "need a candidate list, m_best and T");
    if (K < 1) return fail(ctx, PST_EINVAL, "need K >= 1 (K=%d)", K);
    SweepPlan P;
    if ((rc = plan_sweep(ctx, n, m_list, num_m, l_list, K, &P))) return rc;
    char *ws = (char *)ws_dev;
    int best = -1;
    double best_score = 0.0;
    if (ctx->opt_batched) {
        if (!ws) return fail(ctx, PST_EINVAL, "workspace is NULL");
        if (((uintptr_t)ws & 255) != 0) return fail(ctx, PST_EINVAL, "workspace must be 256-byte aligned");
        if (ws_bytes < P.total)
            return fail(ctx, PST_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, P.total);
        if (ctx->opt_tune_geometry) {  // tile geometry of every length, then the shapes again
            for (size_t j = 0; j < P.ls.size(); ++j)
                HIPCHK(ctx, launch_series_stats(T_dev, ws + P.o_stats[j], P.SL[j], ctx->stream));
            ProfileJob jobs[kMaxJobs];
            const int nj = sweep_jobs(P, ws, P.grid, jobs, 0);
            for (int j = 0; j < nj; ++j) {
                int32_t code = 0;
                float ms = 0.0f;
                if ((rc = tune_geometry_job(ctx, jobs[j], &code, &ms))) return rc;
            }
            sweep_shapes(&P);
        }
        std::vector<double> res;
        if ((rc = run_sweep(ctx, P, T_dev, ws, ws_bytes, m_list, l_list, &res))) return rc;
        const int S = P.out_stride;
        for (int i = 0; i < num_m; ++i)
            if (res[i * S + 2] != 0.0) return fail(ctx, PST_EINVAL, "T holds a non-finite value");
        for (int i = 0; i < num_m; ++i) {
            const uint32_t bits = (uint32_t)res[i * S + 1];
            float dmax;
            std::memcpy(&dmax, &bits, sizeof dmax);
            const double score = dmax > 0.0f ? res[i * S] / (double)dmax : 0.0;
            if (scores_host) scores_host[i] = score;
            if (best < 0 || score > best_score || (score == best_score && m_list[i] < m_list[best])) {
                best = i;
                best_score = score;
            }
        }
        *m_best = m_list[best];
        const Layout &L = P.L[best];
        if (owner_dev || profiles_dev) {
            GreedyJob G = sweep_greedy(P, best, ws);
            G.owner = owner_dev;
            G.profiles = profiles_dev;
            HIPCHK(ctx, launch_owner(G, ctx->stream));
            HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        }
        std::vector<pst_snippet> rec(K);
        for (int p = 0; p < K; ++p) {
            rec[p].segment = (int32_t)res[best * S + 3 + K + p];
            rec[p].greedy_rank = p;
            rec[p].frac = res[best * S + 3 + 2 * K + p] / (double)L.Nm;
            rec[p].area_after = res[best * S + 3 + p];
        }
        std::stable_sort(rec.begin(), rec.end(),
                         [](const pst_snippet &a, const pst_snippet &b) { return a.frac > b.frac; });
        if (out_host) std::memcpy(out_host, rec.data(), sizeof(pst_snippet) * K);
        return PST_OK;
    }
    // one length at a time (the plain path, kept for comparison)
    for (int i = 0; i < num_m; ++i)
        if ((rc = check_ws(ctx, P.L[i], ws_dev, ws_bytes))) return rc;
    for (int i = 0; i < num_m; ++i) {
        if ((rc = snippets_device(ctx, T_dev, P.L[i], ws, nullptr, nullptr, true))) return rc;
        double score = 0.0;
        if ((rc = collect_records(ctx, P.L[i], ws, nullptr, nullptr, &score))) return rc;
        if (scores_host) scores_host[i] = score;
        if (best < 0 || score > best_score || (score == best_score && m_list[i] < m_list[best])) {
            best = i;
            best_score = score;
        }
    }
    *m_best = m_list[best];
    if ((rc = snippets_device(ctx, T_dev, P.L[best], ws, owner_dev, profiles_dev, false))) return rc;
    return collect_records(ctx, P.L[best], ws, out_host, nullptr, nullptr);
}

}  // extern "C"

namespace {
#include "pst_server.inc"
