// Symmetrised graph, weighted Cuthill-McKee, aggregation, quotient graphs and
// expansion: the building blocks of the Band-k ordering (Section 2.2).
#include <algorithm>
#include <numeric>
#include <tuple>

#include "host.hpp"

namespace csrk {

namespace {

// Neighbour / start-vertex sort key: smaller is taken first.
struct Key {
    int64_t a;  // -weight (neighbour key) or -wp (start key)
    int64_t deg;
    int64_t id;
    int32_t v;
    bool operator<(const Key &o) const { return std::tie(a, deg, id) < std::tie(o.a, o.deg, o.id); }
};

}  // namespace

Graph graph_from_csr(int32_t n, const int32_t *row_ptr, const int32_t *col_idx) {
    Graph g;
    g.n = n;
    std::vector<int64_t> cnt(static_cast<size_t>(n) + 1, 0);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            int32_t j = col_idx[k];
            if (j != i) {
                ++cnt[i + 1];
                ++cnt[j + 1];
            }
        }
    std::partial_sum(cnt.begin(), cnt.end(), cnt.begin());
    std::vector<int32_t> raw(static_cast<size_t>(cnt[n]));
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int32_t i = 0; i < n; ++i)
        for (int32_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            int32_t j = col_idx[k];
            if (j != i) {
                raw[fill[i]++] = j;
                raw[fill[j]++] = i;
            }
        }
    g.xadj.assign(static_cast<size_t>(n) + 1, 0);
    g.adj.reserve(raw.size());
    for (int32_t i = 0; i < n; ++i) {
        auto b = raw.begin() + cnt[i], e = raw.begin() + cnt[i + 1];
        std::sort(b, e);
        e = std::unique(b, e);
        g.adj.insert(g.adj.end(), b, e);
        g.xadj[i + 1] = static_cast<int64_t>(g.adj.size());
    }
    g.adj.shrink_to_fit();
    g.wgt.assign(g.adj.size(), 1);
    g.ident.resize(n);
    std::iota(g.ident.begin(), g.ident.end(), 0);
    return g;
}

std::vector<int32_t> cuthill_mckee(const Graph &g) {
    const int32_t n = g.n;
    std::vector<int32_t> starts(n);
    std::iota(starts.begin(), starts.end(), 0);
    std::sort(starts.begin(), starts.end(), [&](int32_t a, int32_t b) {
        return std::make_pair(g.degree(a), g.ident[a]) < std::make_pair(g.degree(b), g.ident[b]);
    });
    std::vector<uint8_t> seen(n, 0);
    std::vector<int32_t> seq;
    seq.reserve(n);
    std::vector<Key> cand;
    for (int32_t s : starts) {
        if (seen[s]) continue;
        seen[s] = 1;
        size_t head = seq.size();
        seq.push_back(s);  // the sequence is the FIFO queue itself
        while (head < seq.size()) {
            int32_t u = seq[head++];
            cand.clear();
            for (int64_t p = g.xadj[u]; p < g.xadj[u + 1]; ++p) {
                int32_t v = g.adj[p];
                if (!seen[v]) cand.push_back({-g.wgt[p], g.degree(v), g.ident[v], v});
            }
            std::sort(cand.begin(), cand.end());
            for (const Key &c : cand) {
                seen[c.v] = 1;
                seq.push_back(c.v);
            }
        }
    }
    return seq;
}

Aggregation aggregate(const Graph &g, int32_t chunk) {
    if (chunk < 1) throw Error{CSRK_ERR_ARG, "group size must be >= 1"};
    std::vector<int32_t> seq = cuthill_mckee(g);
    const int64_t n = g.n;
    const int32_t nc = static_cast<int32_t>((n + chunk - 1) / chunk);
    std::vector<int64_t> cid(nc);
    for (int32_t c = 0; c < nc; ++c) {
        int64_t m = INT64_MAX;
        for (int64_t q = int64_t(c) * chunk; q < std::min(n, int64_t(c + 1) * chunk); ++q) m = std::min(m, g.ident[seq[q]]);
        cid[c] = m;
    }
    std::vector<int32_t> order(nc);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return cid[a] < cid[b]; });
    Aggregation a;
    a.ncoarse = nc;
    a.owner.resize(n);
    a.child_ptr.assign(static_cast<size_t>(nc) + 1, 0);
    a.children.reserve(n);
    a.ident.resize(nc);
    for (int32_t c = 0; c < nc; ++c) {
        int32_t src = order[c];
        int64_t b = int64_t(src) * chunk, e = std::min(n, int64_t(src + 1) * chunk);
        size_t first = a.children.size();
        for (int64_t q = b; q < e; ++q) {
            a.children.push_back(seq[q]);
            a.owner[seq[q]] = c;
        }
        std::sort(a.children.begin() + first, a.children.end());
        a.child_ptr[c + 1] = static_cast<int64_t>(a.children.size());
        a.ident[c] = cid[src];
    }
    return a;
}

Graph quotient(const Graph &g, const Aggregation &a) {
    Graph q;
    q.n = a.ncoarse;
    q.ident = a.ident;
    q.xadj.assign(static_cast<size_t>(q.n) + 1, 0);
    std::vector<int32_t> mark(q.n, -1);
    std::vector<int64_t> acc(q.n, 0);
    std::vector<int32_t> touched;
    for (int32_t c = 0; c < q.n; ++c) {
        touched.clear();
        for (int64_t t = a.child_ptr[c]; t < a.child_ptr[c + 1]; ++t) {
            int32_t u = a.children[t];
            for (int64_t p = g.xadj[u]; p < g.xadj[u + 1]; ++p) {
                int32_t b = a.owner[g.adj[p]];
                if (b == c) continue;
                if (mark[b] != c) {
                    mark[b] = c;
                    acc[b] = 0;
                    touched.push_back(b);
                }
                acc[b] += g.wgt[p];
            }
        }
        std::sort(touched.begin(), touched.end());
        for (int32_t b : touched) {
            q.adj.push_back(b);
            q.wgt.push_back(acc[b]);
        }
        q.xadj[c + 1] = static_cast<int64_t>(q.adj.size());
    }
    return q;
}

std::vector<int32_t> expand(const Graph &g, const std::vector<int32_t> &order_up, const Aggregation &a) {
    const int32_t n = g.n;
    std::vector<int64_t> wp(n, 0);
    std::vector<uint8_t> placed(n, 0);
    std::vector<int32_t> group(n, -1);
    std::vector<int32_t> out;
    out.reserve(n);
    std::vector<int32_t> queue;
    std::vector<Key> cand;
    for (size_t gi = 0; gi < order_up.size(); ++gi) {
        const int32_t up = order_up[gi];
        const int64_t cb = a.child_ptr[up], ce = a.child_ptr[up + 1];
        for (int64_t t = cb; t < ce; ++t) group[a.children[t]] = static_cast<int32_t>(gi);
        int64_t left = ce - cb;
        while (left > 0) {
            int32_t s = -1;
            Key best{};
            for (int64_t t = cb; t < ce; ++t) {
                int32_t v = a.children[t];
                if (placed[v]) continue;
                Key k{-wp[v], g.degree(v), g.ident[v], v};
                if (s < 0 || k < best) {
                    best = k;
                    s = v;
                }
            }
            placed[s] = 1;
            queue.clear();
            queue.push_back(s);
            for (size_t head = 0; head < queue.size(); ++head) {
                int32_t u = queue[head];
                out.push_back(u);
                --left;
                cand.clear();
                for (int64_t p = g.xadj[u]; p < g.xadj[u + 1]; ++p) {
                    int32_t v = g.adj[p];
                    wp[v] += g.wgt[p];
                    if (group[v] == static_cast<int32_t>(gi) && !placed[v])
                        cand.push_back({-g.wgt[p], g.degree(v), g.ident[v], v});
                }
                std::sort(cand.begin(), cand.end());
                for (const Key &c : cand) {
                    placed[c.v] = 1;
                    queue.push_back(c.v);
                }
            }
        }
    }
    return out;
}

namespace {

std::vector<int32_t> running(const std::vector<int64_t> &sizes) {
    std::vector<int32_t> p(sizes.size() + 1, 0);
    for (size_t i = 0; i < sizes.size(); ++i) p[i + 1] = p[i] + static_cast<int32_t>(sizes[i]);
    return p;
}

}  // namespace

Grouping bandk(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, int32_t srs, int32_t ssrs) {
    if (srs < 1 || ssrs < 1) throw Error{CSRK_ERR_ARG, "srs and ssrs must be >= 1"};
    Grouping r;
    if (n == 0) {
        r.sr_ptr = {0};
        r.ssr_ptr = {0};
        return r;
    }
    Graph g0 = graph_from_csr(n, row_ptr, col_idx);
    Aggregation a1 = aggregate(g0, srs);
    Graph g1 = quotient(g0, a1);
    Aggregation a2 = aggregate(g1, ssrs);
    Graph g2 = quotient(g1, a2);
    std::vector<int32_t> order2 = cuthill_mckee(g2);
    std::reverse(order2.begin(), order2.end());
    std::vector<int32_t> order1 = expand(g1, order2, a2);
    r.perm = expand(g0, order1, a1);
    std::vector<int64_t> srsz, ssrsz;
    srsz.reserve(order1.size());
    for (int32_t s : order1) srsz.push_back(a1.child_ptr[s + 1] - a1.child_ptr[s]);
    for (int32_t t : order2) ssrsz.push_back(a2.child_ptr[t + 1] - a2.child_ptr[t]);
    r.sr_ptr = running(srsz);
    r.ssr_ptr = running(ssrsz);
    return r;
}

Grouping bandk_levels(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const std::vector<int32_t> &sizes) {
    if (sizes.empty()) throw Error{CSRK_ERR_ARG, "at least one group size"};
    for (int32_t t : sizes)
        if (t < 1) throw Error{CSRK_ERR_ARG, "group sizes must be >= 1"};
    const size_t levels = sizes.size();
    std::vector<std::vector<int32_t>> ptr(levels, std::vector<int32_t>{0});
    Grouping r;
    if (n > 0) {
        std::vector<Graph> g;
        std::vector<Aggregation> agg;
        g.push_back(graph_from_csr(n, row_ptr, col_idx));
        for (size_t l = 0; l < levels; ++l) {  // coarsen k - 1 times
            agg.push_back(aggregate(g.back(), sizes[l]));
            g.push_back(quotient(g.back(), agg.back()));
        }
        std::vector<int32_t> order = cuthill_mckee(g.back());
        std::reverse(order.begin(), order.end());
        for (size_t l = levels; l >= 1; --l) {  // expand level l into level l - 1
            const Aggregation &a = agg[l - 1];
            std::vector<int64_t> sz;
            sz.reserve(order.size());
            for (int32_t u : order) sz.push_back(a.child_ptr[u + 1] - a.child_ptr[u]);
            ptr[l - 1] = running(sz);
            order = expand(g[l - 1], order, a);
        }
        r.perm = std::move(order);
    }
    r.sr_ptr = std::move(ptr[0]);
    if (levels >= 2) r.ssr_ptr = std::move(ptr[1]);
    for (size_t l = 2; l < levels; ++l) r.upper.push_back(std::move(ptr[l]));
    return r;
}

void chunk_upper(Grouping &g, int32_t k, int32_t t) {
    if (t < 1) throw Error{CSRK_ERR_ARG, "group size must be >= 1"};
    g.upper.clear();
    int64_t units = int64_t(g.ssr_ptr.size()) - 1;
    for (int32_t l = 3; l < k; ++l) {
        std::vector<int64_t> sz;
        for (int64_t u = 0; u < units; u += t) sz.push_back(std::min<int64_t>(t, units - u));
        g.upper.push_back(running(sz));
        units = int64_t(sz.size());
    }
}

Grouping bandk2(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, int32_t srs, int32_t group) {
    if (srs < 1 || group < 1) throw Error{CSRK_ERR_ARG, "srs and ssrs must be >= 1"};
    Grouping r;
    if (n == 0) {
        r.sr_ptr = {0};
        r.ssr_ptr = {0};
        return r;
    }
    Graph g0 = graph_from_csr(n, row_ptr, col_idx);
    Aggregation a1 = aggregate(g0, srs);
    Graph g1 = quotient(g0, a1);
    std::vector<int32_t> order1 = cuthill_mckee(g1);
    std::reverse(order1.begin(), order1.end());
    r.perm = expand(g0, order1, a1);
    std::vector<int64_t> srsz, ssrsz;
    srsz.reserve(order1.size());
    for (int32_t s : order1) srsz.push_back(a1.child_ptr[s + 1] - a1.child_ptr[s]);
    const int64_t nsr = static_cast<int64_t>(srsz.size());
    for (int64_t t = 0; t * group < nsr; ++t) ssrsz.push_back(std::min<int64_t>(group, nsr - t * group));
    r.sr_ptr = running(srsz);
    r.ssr_ptr = running(ssrsz);
    return r;
}

Grouping chunked(std::vector<int32_t> perm, int32_t srs, int32_t ssrs) {
    if (srs < 1 || ssrs < 1) throw Error{CSRK_ERR_ARG, "srs and ssrs must be >= 1"};
    Grouping r;
    const int64_t n = static_cast<int64_t>(perm.size());
    r.perm = std::move(perm);
    std::vector<int64_t> srsz, ssrsz;
    for (int64_t s = 0; s * srs < n; ++s) srsz.push_back(std::min<int64_t>(srs, n - s * srs));
    const int64_t nsr = static_cast<int64_t>(srsz.size());
    for (int64_t t = 0; t * ssrs < nsr; ++t) ssrsz.push_back(std::min<int64_t>(ssrs, nsr - t * ssrs));
    r.sr_ptr = running(srsz);
    r.ssr_ptr = running(ssrsz);
    return r;
}

Grouping rcm_chunked(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, int32_t srs, int32_t ssrs) {
    Graph g0 = graph_from_csr(n, row_ptr, col_idx);
    std::vector<int32_t> order = cuthill_mckee(g0);
    std::reverse(order.begin(), order.end());
    return chunked(std::move(order), srs, ssrs);
}

Grouping from_sizes(std::vector<int32_t> perm, const int32_t *sr_sizes, int32_t nsr, const int32_t *ssr_sizes,
                    int32_t nssr) {
    const int64_t n = static_cast<int64_t>(perm.size());
    if (nsr < 0 || nssr < 0 || (nsr > 0 && !sr_sizes) || (nssr > 0 && !ssr_sizes))
        throw Error{CSRK_ERR_ARG, "bad group size arrays"};
    std::vector<uint8_t> hit(n, 0);
    for (int32_t v : perm) {
        if (v < 0 || v >= n || hit[v]) throw Error{CSRK_ERR_ARG, "perm is not a permutation of 0..n-1"};
        hit[v] = 1;
    }
    std::vector<int64_t> a(sr_sizes, sr_sizes + nsr), b(ssr_sizes, ssr_sizes + nssr);
    int64_t tot = 0;
    for (int64_t s : a) {
        if (s < 1) throw Error{CSRK_ERR_ARG, "super-row sizes must be >= 1"};
        tot += s;
    }
    if (tot != n) throw Error{CSRK_ERR_ARG, "super-row sizes must add up to n"};
    tot = 0;
    for (int64_t s : b) {
        if (s < 1) throw Error{CSRK_ERR_ARG, "super-super-row sizes must be >= 1"};
        tot += s;
    }
    if (tot != nsr) throw Error{CSRK_ERR_ARG, "super-super-row sizes must add up to nsr"};
    Grouping r;
    r.perm = std::move(perm);
    r.sr_ptr = running(a);
    r.ssr_ptr = running(b);
    return r;
}

int64_t sr_budget(int32_t n, int64_t nnz, int32_t srs) {
    if (n <= 0) return 2048;
    const int64_t q = (4 * int64_t(srs) * nnz + n - 1) / n;
    return std::max<int64_t>(2048, q);
}

void balance(Grouping &g, const int32_t *row_ptr, int64_t budget, int32_t ssrs) {
    const int64_t nsr = int64_t(g.sr_ptr.size()) - 1;
    if (nsr <= 0) return;
    auto cost = [&](int32_t i) -> int64_t {
        const int32_t r = g.perm[i];
        const int64_t len = int64_t(row_ptr[r + 1]) - row_ptr[r];
        return len > CSRK_LONG_ROW ? 0 : len;
    };
    std::vector<int64_t> sr_sizes, ssr_sizes;
    sr_sizes.reserve(size_t(nsr));
    bool split_any = false;
    for (size_t t = 0; t + 1 < g.ssr_ptr.size(); ++t) {
        const size_t first = sr_sizes.size();
        for (int32_t s = g.ssr_ptr[t]; s < g.ssr_ptr[t + 1]; ++s) {
            const int32_t a = g.sr_ptr[s], b = g.sr_ptr[s + 1];
            int64_t total = 0;
            for (int32_t i = a; i < b; ++i) total += cost(i);
            if (total <= budget) {
                sr_sizes.push_back(b - a);
                continue;
            }
            split_any = true;
            int32_t start = a;
            int64_t acc = 0;
            for (int32_t i = a; i < b; ++i) {
                const int64_t c = cost(i);
                if (i > start && acc + c > budget) {
                    sr_sizes.push_back(i - start);
                    start = i;
                    acc = 0;
                }
                acc += c;
            }
            sr_sizes.push_back(b - start);
        }
        const int32_t pieces = static_cast<int32_t>(sr_sizes.size() - first);
        for (int32_t q = 0; q < pieces; q += ssrs) ssr_sizes.push_back(std::min<int64_t>(ssrs, pieces - q));
    }
    if (!split_any) return;
    // rows where each level-3 unit starts, to recount it over the new SSRs
    std::vector<int32_t> start_rows;
    if (!g.upper.empty())
        for (int32_t u : g.upper[0]) start_rows.push_back(g.sr_ptr[g.ssr_ptr[u]]);
    g.sr_ptr = running(sr_sizes);
    g.ssr_ptr = running(ssr_sizes);
    size_t t = 0;
    for (size_t q = 0; q < start_rows.size(); ++q) {
        while (g.sr_ptr[g.ssr_ptr[t]] < start_rows[q]) ++t;  // the new SSR that starts at this row
        g.upper[0][q] = static_cast<int32_t>(t);
    }
}

}  // namespace csrk
