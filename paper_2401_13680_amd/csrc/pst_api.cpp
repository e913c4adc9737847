// Host runtime behind include/pst.h: argument validation, workspace layout,
// launch sequencing on the caller's stream, and the host-side tail of the
// snippet search (ordering K records by frac, eq. 8).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <vector>

#include "../../include/pst.h"
#include "pst_internal.h"

struct pst_ctx {
    int device;
    hipStream_t stream;
    bool poisoned;
    bool timing;
    bool timed;
    hipEvent_t ev0, ev1;
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
int plan(pst_ctx *c, int64_t n, int32_t m, int32_t l, int32_t k, int32_t K, Layout *L) {
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
    L->grid = profile_grid(L->ntile * nseg);
    L->nblk = (int32_t)((L->Nm + kSumBlock - 1) / kSumBlock);
    L->nblk2 = (int32_t)std::min<int64_t>(1024, (L->Nm + 255) / 256);
    L->sT = stats_layout(n, l);
    L->sQ = stats_layout(m, l);
    size_t o = 0;
    L->o_T = o;      o = al(o + L->sT.total);
    L->o_Q = o;      o = al(o + L->sQ.total);
    L->o_rw = o;     o = al(o + sizeof(float) * profile_scratch_floats(L->grid, w));
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
hipError_t timed_profile(pst_ctx *c, const ProfileJob &j) {
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
    c->err[0] = 0;
    *out = c;
    return PST_OK;
}

void pst_destroy(pst_ctx *ctx) {
    if (!ctx) return;
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
    if (!m_list || num_m < 1) return 0;
    size_t mx = 0;
    for (int i = 0; i < num_m; ++i) {
        const int32_t l = l_list ? l_list[i] : m_list[i] / 2;
        const size_t b = pst_workspace_bytes(n, m_list[i], l, K);
        if (b == 0) return 0;
        mx = std::max(mx, b);
    }
    return mx;
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
    j.grid = profile_grid(L.ntile);
    HIPCHK(ctx, timed_profile(ctx, j));
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

int pst_select_length(pst_ctx *ctx, const double *T_dev, int64_t n, const int32_t *m_list,
                      int32_t num_m, const int32_t *l_list, int32_t K, int32_t *m_best,
                      double *scores_host, pst_snippet *out_host, float *profiles_dev,
                      int32_t *owner_dev, void *ws_dev, size_t ws_bytes) {
    int rc = begin(ctx);
    if (rc) return rc;
    if (!m_list || num_m < 1 || !m_best || !T_dev)
        return fail(ctx, PST_EINVAL, "need a candidate list, m_best and T");
    if (K < 1) return fail(ctx, PST_EINVAL, "need K >= 1 (K=%d)", K);
    std::vector<Layout> Ls(num_m);
    for (int i = 0; i < num_m; ++i) {
        const int32_t l = l_list ? l_list[i] : m_list[i] / 2;
        if ((rc = plan(ctx, n, m_list[i], l, 0, K, &Ls[i]))) return rc;
        if ((rc = check_ws(ctx, Ls[i], ws_dev, ws_bytes))) return rc;
    }
    char *ws = (char *)ws_dev;
    int best = -1;
    double best_score = 0.0;
    for (int i = 0; i < num_m; ++i) {
        if ((rc = snippets_device(ctx, T_dev, Ls[i], ws, nullptr, nullptr, true))) return rc;
        double score = 0.0;
        if ((rc = collect_records(ctx, Ls[i], ws, nullptr, nullptr, &score))) return rc;
        if (scores_host) scores_host[i] = score;
        if (best < 0 || score > best_score || (score == best_score && m_list[i] < m_list[best])) {
            best = i;
            best_score = score;
        }
    }
    *m_best = m_list[best];
    if ((rc = snippets_device(ctx, T_dev, Ls[best], ws, owner_dev, profiles_dev, false))) return rc;
    return collect_records(ctx, Ls[best], ws, out_host, nullptr, nullptr);
}

}  // extern "C"
