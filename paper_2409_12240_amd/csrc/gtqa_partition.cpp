// Host-side balanced bipartition for the mean-field entanglement entropy
// (Sec. III.C, Eq. bipartition): spectral partitioning.  The Fiedler vector
// of the graph Laplacian L = D - Adj (the eigenvector of its second smallest
// eigenvalue, the relaxation of the ratio cut |dA| / (|A| |A-bar|)) orders
// the vertices; the best prefix of that order under the same ratio is A.
//
// The eigenvector comes from Lanczos iterations with full
// reorthogonalisation on the complement of the constant vector, restarted
// from the current Ritz vector until its residual is small; the smallest
// eigenpair of each tridiagonal matrix is found by Sturm-sequence bisection
// and inverse iteration.

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <numeric>
#include <vector>

#include "gtqa.h"

namespace {

struct Graph {
    int n = 0;
    std::vector<std::vector<int>> nbr;
};

// y = L x
void laplacian_apply(const Graph& g, const std::vector<double>& x, std::vector<double>& y) {
    for (int a = 0; a < g.n; ++a) {
        double s = (double)g.nbr[a].size() * x[a];
        for (int b : g.nbr[a]) s -= x[b];
        y[a] = s;
    }
}

double dot(const std::vector<double>& a, const std::vector<double>& b) {
    double s = 0.0;
    for (size_t i = 0; i < a.size(); ++i) s += a[i] * b[i];
    return s;
}

// removes the component along the constant vector, then normalises
bool center_normalise(std::vector<double>& x) {
    const double mean = std::accumulate(x.begin(), x.end(), 0.0) / (double)x.size();
    for (double& v : x) v -= mean;
    const double nr = std::sqrt(dot(x, x));
    if (!(nr > 0.0)) return false;
    for (double& v : x) v /= nr;
    return true;
}

// number of eigenvalues below s of the symmetric tridiagonal matrix with
// diagonal a and off-diagonal b (LDL^T pivots of T - s I)
int sturm_count(const std::vector<double>& a, const std::vector<double>& b, double s) {
    int cnt = 0;
    double q = 1.0;
    for (size_t i = 0; i < a.size(); ++i) {
        const double off = i ? b[i - 1] * b[i - 1] / q : 0.0;
        q = a[i] - s - off;
        if (q == 0.0) q = -1e-300;
        if (q < 0.0) ++cnt;
    }
    return cnt;
}

// smallest eigenpair of the tridiagonal (a, b): bisection, then inverse iteration
double smallest_eigenpair(const std::vector<double>& a, const std::vector<double>& b, std::vector<double>& y) {
    const size_t k = a.size();
    double lo = a[0], hi = a[0];
    for (size_t i = 0; i < k; ++i) {
        const double r = (i ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < k ? std::fabs(b[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    for (int it = 0; it < 200 && hi - lo > 1e-15 * std::max(1.0, std::fabs(hi)); ++it) {
        const double mid = 0.5 * (lo + hi);
        if (sturm_count(a, b, mid) >= 1) hi = mid;
        else lo = mid;
    }
    const double theta = hi;
    // inverse iteration on T - (theta - delta) I by the tridiagonal recurrence
    const double shift = theta - 1e-12 * std::max(1.0, std::fabs(theta));
    y.assign(k, 1.0);
    std::vector<double> c(k), d(k);
    for (int it = 0; it < 4; ++it) {
        // forward elimination
        double piv = a[0] - shift;
        c[0] = (k > 1 ? b[0] : 0.0) / piv;
        d[0] = y[0] / piv;
        for (size_t i = 1; i < k; ++i) {
            piv = a[i] - shift - b[i - 1] * c[i - 1];
            if (piv == 0.0) piv = 1e-300;
            c[i] = (i + 1 < k ? b[i] : 0.0) / piv;
            d[i] = (y[i] - b[i - 1] * d[i - 1]) / piv;
        }
        y[k - 1] = d[k - 1];
        for (size_t i = k - 1; i-- > 0;) y[i] = d[i] - c[i] * y[i + 1];
        const double nr = std::sqrt(dot(y, y));
        for (double& v : y) v /= nr;
    }
    return theta;
}

// Fiedler vector of the graph's Laplacian (unit norm, orthogonal to 1)
bool fiedler_vector(const Graph& g, std::vector<double>& x) {
    const int n = g.n;
    const int kmax = std::min(n - 1, 160);
    x.resize(n);
    for (int a = 0; a < n; ++a) x[a] = std::cos(1.2345 * a + 0.5) + 1e-3 * (a % 7);
    if (!center_normalise(x)) return false;
    std::vector<std::vector<double>> Q;
    std::vector<double> w(n), y;
    for (int restart = 0; restart < 12; ++restart) {
        Q.assign(1, x);
        std::vector<double> al, be;
        for (int j = 0; j < kmax; ++j) {
            laplacian_apply(g, Q[j], w);
            const double aj = dot(w, Q[j]);
            al.push_back(aj);
            // full reorthogonalisation (twice) against the basis and the constant vector
            for (int pass = 0; pass < 2; ++pass) {
                for (const auto& q : Q) {
                    const double h = dot(w, q);
                    for (int i = 0; i < n; ++i) w[i] -= h * q[i];
                }
                const double mean = std::accumulate(w.begin(), w.end(), 0.0) / n;
                for (double& v : w) v -= mean;
            }
            const double bj = std::sqrt(dot(w, w));
            if (j + 1 == kmax || bj < 1e-12) break;
            be.push_back(bj);
            for (double& v : w) v /= bj;
            Q.push_back(w);
        }
        be.resize(al.size() > 0 ? al.size() - 1 : 0);
        const double theta = smallest_eigenpair(al, be, y);
        std::fill(x.begin(), x.end(), 0.0);
        for (size_t i = 0; i < y.size(); ++i)
            for (int a = 0; a < n; ++a) x[a] += y[i] * Q[i][a];
        if (!center_normalise(x)) return false;
        laplacian_apply(g, x, w);
        double res = 0.0;
        for (int a = 0; a < n; ++a) res += (w[a] - theta * x[a]) * (w[a] - theta * x[a]);
        if (std::sqrt(res) < 1e-10 * std::max(1.0, theta)) break;
    }
    return true;
}

}  // namespace

extern "C" int gtqa_spectral_bipartition(int32_t n, int32_t n_edges, const int32_t* edges, uint8_t* side_out,
                                         int32_t* cut_out) {
    if (n < 2 || n_edges < 0 || (n_edges > 0 && !edges) || !side_out) return GTQA_ERR_ARG;
    Graph g;
    g.n = n;
    g.nbr.assign(n, {});
    for (int e = 0; e < n_edges; ++e) {
        const int u = edges[2 * e], v = edges[2 * e + 1];
        if (u < 0 || v < 0 || u >= n || v >= n || u == v) return GTQA_ERR_GRAPH;
        g.nbr[u].push_back(v);
        g.nbr[v].push_back(u);
    }
    std::vector<double> f;
    if (!fiedler_vector(g, f)) return GTQA_ERR_NUMERIC;
    // sign: the entry of largest magnitude (first on ties) is positive
    int imax = 0;
    for (int a = 1; a < n; ++a)
        if (std::fabs(f[a]) > std::fabs(f[imax])) imax = a;
    if (f[imax] < 0.0)
        for (double& v : f) v = -v;
    std::vector<int> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return f[a] < f[b]; });
    // sweep the prefixes of the order, keeping the cut size incrementally
    std::vector<uint8_t> in(n, 0);
    long cut = 0;
    double best = INFINITY;
    int bestk = 0;
    long bestcut = 0;
    for (int k = 1; k < n; ++k) {
        const int a = order[k - 1];
        for (int b : g.nbr[a]) cut += in[b] ? -1 : 1;
        in[a] = 1;
        const double r = (double)cut / ((double)k * (double)(n - k));
        if (r < best) {
            best = r;
            bestk = k;
            bestcut = cut;
        }
    }
    for (int a = 0; a < n; ++a) side_out[a] = 0;
    for (int k = 0; k < bestk; ++k) side_out[order[k]] = 1;
    if (cut_out) *cut_out = (int32_t)bestcut;
    return GTQA_OK;
}
