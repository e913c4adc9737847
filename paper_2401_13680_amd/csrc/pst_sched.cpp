// Scheduling of section 4.2: run times predicted by polynomial regression on
// earlier runs, and the Karmarkar-Karp largest-differencing partition that
// spreads the candidate lengths over workers with balanced predicted load.
// Host code only (no device work).
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <queue>
#include <vector>

#include "../../include/pst.h"
#include "pst_sched.h"

namespace {

// The three sizes that set a run's work, scaled to order one: segments n/m
// (in thousands), window width w = m-l+1 (in hundreds), subsequences n-l+1
// (in units of 10^5).  The distance-matrix cell count is their product.
bool scaled_sizes(int64_t n, int32_t m, int32_t l, double *u, double *w, double *v) {
    if (m < 2 || l < 2 || l > m || n < m) return false;
    *u = (double)(n / m) / 1e3;
    *w = (double)(m - l + 1) / 1e2;
    *v = (double)(n - l + 1) / 1e5;
    return true;
}

double ipow(double x, int e) {
    double r = 1.0;
    for (int i = 0; i < e; ++i) r *= x;
    return r;
}

// Monomials u^a w^b v^c of total degree t = 0..D, for each t with a from t
// down to 0 and b from t-a down to 0 (c = t-a-b).
void monomials(int D, double u, double w, double v, std::vector<double> &f) {
    f.clear();
    for (int t = 0; t <= D; ++t)
        for (int a = t; a >= 0; --a)
            for (int b = t - a; b >= 0; --b) f.push_back(ipow(u, a) * ipow(w, b) * ipow(v, t - a - b));
}

int num_monomials(int D) { return (D + 1) * (D + 2) * (D + 3) / 6; }

// Least squares min |A c - y| by Householder QR (A: rows x cols, row-major,
// rows >= cols, full column rank); false when a column is (numerically) zero.
bool lstsq_qr(std::vector<double> A, std::vector<double> y, int rows, int cols, std::vector<double> &c) {
    for (int j = 0; j < cols; ++j) {
        double nrm = 0.0;
        for (int i = j; i < rows; ++i) nrm += A[(size_t)i * cols + j] * A[(size_t)i * cols + j];
        nrm = std::sqrt(nrm);
        if (nrm == 0.0) return false;
        const double a0 = A[(size_t)j * cols + j];
        const double alpha = a0 > 0 ? -nrm : nrm;
        // v = x - alpha e1, stored in place below the diagonal
        std::vector<double> hv(rows - j);
        for (int i = j; i < rows; ++i) hv[i - j] = A[(size_t)i * cols + j];
        hv[0] -= alpha;
        double vv = 0.0;
        for (double t : hv) vv += t * t;
        if (vv == 0.0) continue;
        for (int k = j; k < cols; ++k) {
            double s = 0.0;
            for (int i = j; i < rows; ++i) s += hv[i - j] * A[(size_t)i * cols + k];
            s = 2.0 * s / vv;
            for (int i = j; i < rows; ++i) A[(size_t)i * cols + k] -= s * hv[i - j];
        }
        double s = 0.0;
        for (int i = j; i < rows; ++i) s += hv[i - j] * y[i];
        s = 2.0 * s / vv;
        for (int i = j; i < rows; ++i) y[i] -= s * hv[i - j];
    }
    c.assign(cols, 0.0);
    for (int j = cols - 1; j >= 0; --j) {
        double s = y[j];
        for (int k = j + 1; k < cols; ++k) s -= A[(size_t)j * cols + k] * c[k];
        const double d = A[(size_t)j * cols + j];
        if (d == 0.0) return false;
        c[j] = s / d;
    }
    return true;
}

// k-way largest differencing.  Every item starts as a k-tuple (cost, 0, ..,
// 0); the two tuples of largest spread (max - min; ties to the older tuple)
// are merged slot by slot, the largest slot of one with the smallest of the
// other, and the merged slots are re-sorted largest first (stable), until one
// tuple is left: its slots are the parts.
struct Tup {
    std::vector<double> s;               // slot sums, largest first
    std::vector<std::vector<int>> items; // items per slot
    int id;
    double spread() const { return s.front() - s.back(); }
};

struct ByLargestSpread {
    const std::vector<Tup> *T;
    bool operator()(int a, int b) const {  // true when a ranks below b
        const double sa = (*T)[a].spread(), sb = (*T)[b].spread();
        if (sa != sb) return sa < sb;
        return (*T)[a].id > (*T)[b].id;
    }
};

void kk(const double *cost, int count, int parts, int *part_out, double *load_out) {
    std::vector<Tup> T;
    T.reserve(2 * (size_t)count);
    for (int i = 0; i < count; ++i) {
        Tup t;
        t.s.assign(parts, 0.0);
        t.items.assign(parts, {});
        t.s[0] = cost[i];
        t.items[0].push_back(i);
        t.id = i;
        T.push_back(std::move(t));
    }
    std::priority_queue<int, std::vector<int>, ByLargestSpread> q(ByLargestSpread{&T});
    for (int i = 0; i < count; ++i) q.push(i);
    int next_id = count;
    while (q.size() > 1) {
        const int a = q.top();
        q.pop();
        const int b = q.top();
        q.pop();
        Tup m;
        m.s.resize(parts);
        m.items.resize(parts);
        for (int j = 0; j < parts; ++j) {
            m.s[j] = T[a].s[j] + T[b].s[parts - 1 - j];
            m.items[j] = T[a].items[j];
            m.items[j].insert(m.items[j].end(), T[b].items[parts - 1 - j].begin(), T[b].items[parts - 1 - j].end());
        }
        std::vector<int> ord(parts);
        for (int j = 0; j < parts; ++j) ord[j] = j;
        std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return m.s[x] > m.s[y]; });
        Tup r;
        r.id = next_id++;
        for (int j : ord) {
            r.s.push_back(m.s[j]);
            r.items.push_back(std::move(m.items[j]));
        }
        T.push_back(std::move(r));
        q.push((int)T.size() - 1);
    }
    for (int j = 0; j < parts; ++j) load_out[j] = 0.0;
    if (q.empty()) return;
    const Tup &f = T[q.top()];
    for (int j = 0; j < parts; ++j) {
        load_out[j] = f.s[j];
        for (int i : f.items[j]) part_out[i] = j;
    }
}

}  // namespace

extern "C" {

int pst_model_create(pst_model **out, int32_t degree) {
    if (!out) return PST_EINVAL;
    *out = nullptr;
    if (degree < 1 || degree > 4) return PST_EINVAL;
    pst_model *M = new pst_model;
    M->degree = degree;
    *out = M;
    return PST_OK;
}

void pst_model_destroy(pst_model *model) { delete model; }

int pst_model_observe(pst_model *M, int64_t n, int32_t m, int32_t l, double ms) {
    double u, w, v;
    if (!M || !scaled_sizes(n, m, l, &u, &w, &v) || !(ms > 0.0) || !std::isfinite(ms)) return PST_EINVAL;
    M->u.push_back(u);
    M->w.push_back(w);
    M->v.push_back(v);
    M->ms.push_back(ms);
    M->fitted = false;
    return PST_OK;
}

int pst_model_fit(pst_model *M) {
    if (!M) return PST_EINVAL;
    const int P = num_monomials(M->degree);
    const int N = (int)M->ms.size();
    if (N < 1) return PST_ENOTREADY;
    // relative least squares (row i weighted by 1/ms_i), plus a ridge of
    // 1e-10 times the mean squared column norm, solved as one augmented
    // least-squares problem: determined even with fewer runs than monomials
    std::vector<double> A((size_t)(N + P) * P, 0.0), y(N + P, 0.0), f;
    double fro = 0.0;
    for (int i = 0; i < N; ++i) {
        monomials(M->degree, M->u[i], M->w[i], M->v[i], f);
        for (int j = 0; j < P; ++j) {
            A[(size_t)i * P + j] = f[j] / M->ms[i];
            fro += A[(size_t)i * P + j] * A[(size_t)i * P + j];
        }
        y[i] = 1.0;
    }
    const double lam = std::sqrt(1e-10 * fro / P);
    for (int j = 0; j < P; ++j) A[(size_t)(N + j) * P + j] = lam;
    std::vector<double> c;
    if (!lstsq_qr(A, y, N + P, P, c)) return PST_EINVAL;
    M->coef = c;
    M->fitted = true;
    return PST_OK;
}

int pst_model_coefficients(const pst_model *M, double *coef_out, int32_t cap, int32_t *num_out) {
    if (!M || !num_out) return PST_EINVAL;
    if (!M->fitted) return PST_ENOTREADY;
    *num_out = (int32_t)M->coef.size();
    if (coef_out)
        for (int j = 0; j < (int)M->coef.size() && j < cap; ++j) coef_out[j] = M->coef[j];
    return PST_OK;
}

int pst_model_predict(const pst_model *M, int64_t n, int32_t m, int32_t l, double *ms_out) {
    double u, w, v;
    if (!M || !ms_out || !scaled_sizes(n, m, l, &u, &w, &v)) return PST_EINVAL;
    if (!M->fitted) return PST_ENOTREADY;
    std::vector<double> f;
    monomials(M->degree, u, w, v, f);
    double s = 0.0;
    for (size_t j = 0; j < f.size(); ++j) s += M->coef[j] * f[j];
    *ms_out = s;
    return PST_OK;
}

int pst_partition_kk(const double *cost, int32_t count, int32_t parts, int32_t *part_out, double *load_out) {
    if (count < 0 || parts < 1 || parts > 4096 || (count > 0 && (!cost || !part_out)) || !load_out)
        return PST_EINVAL;
    if ((int64_t)count * parts > ((int64_t)1 << 24)) return PST_EINVAL;  // the tuples take count * parts slots
    for (int i = 0; i < count; ++i)
        if (!(cost[i] >= 0.0) || !std::isfinite(cost[i])) return PST_EINVAL;
    std::vector<int> po(count);
    kk(cost, count, parts, po.data(), load_out);
    for (int i = 0; i < count; ++i) part_out[i] = po[i];
    return PST_OK;
}

int pst_partition_lengths(const pst_model *M, int64_t n, const int32_t *m_list, const int32_t *l_list,
                          int32_t num_m, int32_t parts, int32_t *part_out, double *load_out) {
    if (!M || !m_list || num_m < 1 || !part_out || !load_out) return PST_EINVAL;
    std::vector<double> cost(num_m);
    for (int i = 0; i < num_m; ++i) {
        const int rc = pst_model_predict(M, n, m_list[i], l_list ? l_list[i] : m_list[i] / 2, &cost[i]);
        if (rc) return rc;
        cost[i] = std::max(cost[i], 0.0);
    }
    return pst_partition_kk(cost.data(), num_m, parts, part_out, load_out);
}

}  // extern "C"
