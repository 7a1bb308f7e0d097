// symbolic.cpp -- nested-dissection ordering and front tree for the
// multifrontal LU of H - sigma.
//
// The paper factors H - E with a parallel sparse LU (section "Numerical
// method") and notes that the Hilbert-space graph of Eq. (1) has a coordination
// number growing like L (the Bethe-lattice paragraph of "Results and finite
// size scaling analysis"), so fill control decides the cost.  This file orders
// the sector graph by recursive vertex bisection (nested dissection, George
// 1973) with multilevel partitions: heavy-edge matching coarsening, greedy
// graph growing on the coarsest graph, Fiduccia-Mattheyses refinement on every
// level, and a minimum vertex cover of the cut edges (Hopcroft-Karp matching +
// Koenig's theorem) turning the edge cut into a vertex separator.  Every
// dissection node becomes one dense front: a leaf subdomain or a separator is
// factored as one dense pivot block (relaxed supernode), which is what lets the
// device factor and solve with dense tiles.
#include "symbolic.hpp"

#include <algorithm>
#include <chrono>
#include <numeric>
#include <queue>
#include <stdexcept>

namespace mbl {
namespace {

struct Rng {
    uint64_t s;
    explicit Rng(uint64_t seed) : s(seed) {}
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ULL);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        return z ^ (z >> 31);
    }
    int below(int n) { return (int)(next() % (uint64_t)n); }
};

struct Graph {
    int n = 0;
    std::vector<int> xadj, adj, ew, vw;
    int64_t total() const {
        int64_t t = 0;
        for (int w : vw) t += w;
        return t;
    }
};

Graph induced(const Graph &g, const std::vector<int> &part, int which, std::vector<int> &sub2g) {
    std::vector<int> g2sub(g.n, -1);
    sub2g.clear();
    for (int v = 0; v < g.n; v++)
        if (part[v] == which) { g2sub[v] = (int)sub2g.size(); sub2g.push_back(v); }
    Graph s;
    s.n = (int)sub2g.size();
    s.xadj.assign(s.n + 1, 0);
    s.vw.resize(s.n);
    for (int i = 0; i < s.n; i++) {
        int v = sub2g[i];
        s.vw[i] = g.vw[v];
        for (int e = g.xadj[v]; e < g.xadj[v + 1]; e++) {
            int u = g2sub[g.adj[e]];
            if (u >= 0) { s.adj.push_back(u); s.ew.push_back(g.ew[e]); }
        }
        s.xadj[i + 1] = (int)s.adj.size();
    }
    return s;
}

// heavy-edge matching; returns the coarse graph and the fine->coarse map
Graph coarsen(const Graph &g, Rng &rng, std::vector<int> &cmap) {
    int n = g.n;
    std::vector<int> match(n, -1), order(n);
    std::iota(order.begin(), order.end(), 0);
    for (int i = n - 1; i > 0; i--) std::swap(order[i], order[rng.below(i + 1)]);
    for (int v : order) {
        if (match[v] != -1) continue;
        int best = -1, bw = -1;
        for (int e = g.xadj[v]; e < g.xadj[v + 1]; e++) {
            int u = g.adj[e];
            if (u != v && match[u] == -1 && g.ew[e] > bw) { best = u; bw = g.ew[e]; }
        }
        if (best < 0) match[v] = v;
        else { match[v] = best; match[best] = v; }
    }
    cmap.assign(n, -1);
    int cn = 0;
    std::vector<int> first, second;
    for (int v = 0; v < n; v++) {
        if (cmap[v] != -1) continue;
        cmap[v] = cn;
        first.push_back(v);
        second.push_back(match[v] != v ? match[v] : -1);
        if (match[v] != v) cmap[match[v]] = cn;
        cn++;
    }
    Graph c;
    c.n = cn;
    c.xadj.assign(cn + 1, 0);
    c.vw.assign(cn, 0);
    std::vector<int> mark(cn, -1), pos(cn, 0);
    for (int cv = 0; cv < cn; cv++) {
        int parts[2] = {first[cv], second[cv]};
        for (int q = 0; q < 2; q++) {
            int v = parts[q];
            if (v < 0) continue;
            c.vw[cv] += g.vw[v];
            for (int e = g.xadj[v]; e < g.xadj[v + 1]; e++) {
                int cu = cmap[g.adj[e]];
                if (cu == cv) continue;
                if (mark[cu] != cv) {
                    mark[cu] = cv;
                    pos[cu] = (int)c.adj.size();
                    c.adj.push_back(cu);
                    c.ew.push_back(g.ew[e]);
                } else {
                    c.ew[pos[cu]] += g.ew[e];
                }
            }
        }
        c.xadj[cv + 1] = (int)c.adj.size();
    }
    return c;
}

int64_t cut_of(const Graph &g, const std::vector<int> &part) {
    int64_t cut = 0;
    for (int v = 0; v < g.n; v++)
        for (int e = g.xadj[v]; e < g.xadj[v + 1]; e++)
            if (part[v] != part[g.adj[e]]) cut += g.ew[e];
    return cut / 2;
}

// Fiduccia-Mattheyses 2-way refinement of an edge cut under weight limits.
void fm_refine(const Graph &g, std::vector<int> &part, const int64_t maxw[2], int passes) {
    int n = g.n;
    std::vector<int64_t> gain(n);
    std::vector<int> stamp(n, 0);
    std::vector<char> locked(n);
    int64_t pw[2] = {0, 0};
    for (int v = 0; v < n; v++) pw[part[v]] += g.vw[v];
    auto compute_gains = [&]() {
        for (int v = 0; v < n; v++) {
            int64_t ext = 0, in = 0;
            for (int e = g.xadj[v]; e < g.xadj[v + 1]; e++)
                (part[g.adj[e]] == part[v] ? in : ext) += g.ew[e];
            gain[v] = ext - in;
        }
    };
    typedef std::pair<int64_t, std::pair<int, int>> Item;  // gain, (stamp, v)
    for (int pass = 0; pass < passes; pass++) {
        compute_gains();
        int64_t cut = cut_of(g, part);
        std::fill(locked.begin(), locked.end(), 0);
        std::priority_queue<Item> pq[2];
        for (int v = 0; v < n; v++) {
            bool bnd = false;
            for (int e = g.xadj[v]; e < g.xadj[v + 1] && !bnd; e++) bnd = part[g.adj[e]] != part[v];
            if (bnd) pq[part[v]].push({gain[v], {stamp[v], v}});
        }
        std::vector<int> moves;
        int64_t best_cut = cut;
        int64_t best_imb = std::llabs(pw[0] - pw[1]);
        size_t best_len = 0;
        size_t limit = std::max<size_t>(64, (size_t)n / 50);
        while (true) {
            int cand[2] = {-1, -1};
            for (int s = 0; s < 2; s++) {
                while (!pq[s].empty()) {
                    auto it = pq[s].top();
                    int v = it.second.second;
                    if (locked[v] || part[v] != s || it.second.first != stamp[v]) { pq[s].pop(); continue; }
                    if (pw[1 - s] + g.vw[v] > maxw[1 - s]) break;  // would overload the target side
                    cand[s] = v;
                    break;
                }
            }
            int s;
            if (cand[0] < 0 && cand[1] < 0) break;
            else if (cand[0] < 0) s = 1;
            else if (cand[1] < 0) s = 0;
            else if (gain[cand[0]] != gain[cand[1]]) s = gain[cand[0]] > gain[cand[1]] ? 0 : 1;
            else s = pw[0] >= pw[1] ? 0 : 1;
            int v = cand[s];
            pq[s].pop();
            part[v] = 1 - s;
            pw[s] -= g.vw[v];
            pw[1 - s] += g.vw[v];
            cut -= gain[v];
            gain[v] = -gain[v];
            locked[v] = 1;
            moves.push_back(v);
            for (int e = g.xadj[v]; e < g.xadj[v + 1]; e++) {
                int u = g.adj[e];
                if (locked[u]) continue;
                gain[u] += (part[u] == part[v]) ? -2 * (int64_t)g.ew[e] : 2 * (int64_t)g.ew[e];
                stamp[u]++;
                pq[part[u]].push({gain[u], {stamp[u], u}});
            }
            int64_t imb = std::llabs(pw[0] - pw[1]);
            if (cut < best_cut || (cut == best_cut && imb < best_imb)) {
                best_cut = cut; best_imb = imb; best_len = moves.size();
            }
            if (moves.size() - best_len > limit) break;
        }
        for (size_t i = moves.size(); i > best_len; i--) {
            int v = moves[i - 1];
            pw[part[v]] -= g.vw[v];
            part[v] = 1 - part[v];
            pw[part[v]] += g.vw[v];
        }
        if (best_len == 0) break;
    }
}

// greedy graph growing from a random seed until half the weight is reached
void grow_bisection(const Graph &g, Rng &rng, int64_t target0, std::vector<int> &part) {
    int n = g.n;
    part.assign(n, 1);
    std::vector<int64_t> conn(n, 0);   // edge weight into part 0
    std::vector<int> stamp(n, 0);
    std::priority_queue<std::pair<int64_t, std::pair<int, int>>> pq;
    int64_t w0 = 0;
    int added = 0;
    while (w0 < target0 && added < n) {
        int v = -1;
        while (!pq.empty()) {
            auto it = pq.top();
            pq.pop();
            int u = it.second.second;
            if (part[u] == 1 && it.second.first == stamp[u]) { v = u; break; }
        }
        if (v < 0) {                       // start (or restart in another component)
            int tries = 0;
            do { v = rng.below(n); } while (part[v] == 0 && ++tries < 4 * n);
            if (part[v] == 0)
                for (v = 0; v < n && part[v] == 0; v++) {}
            if (v >= n) break;
        }
        part[v] = 0;
        w0 += g.vw[v];
        added++;
        for (int e = g.xadj[v]; e < g.xadj[v + 1]; e++) {
            int u = g.adj[e];
            if (part[u] != 1) continue;
            conn[u] += g.ew[e];
            int64_t deg = 0;
            for (int f = g.xadj[u]; f < g.xadj[u + 1]; f++) deg += g.ew[f];
            stamp[u]++;
            pq.push({2 * conn[u] - deg, {stamp[u], u}});
        }
    }
}

// edge bisection of g by the multilevel scheme; part[v] in {0, 1}
void multilevel_bisect(const Graph &g, const NdOptions &opt, Rng &rng, std::vector<int> &part) {
    std::vector<Graph> levels;
    std::vector<std::vector<int>> maps;
    levels.push_back(g);
    while (levels.back().n > 120) {
        std::vector<int> cmap;
        Graph c = coarsen(levels.back(), rng, cmap);
        if (c.n > 0.9 * levels.back().n) break;
        maps.push_back(std::move(cmap));
        levels.push_back(std::move(c));
    }
    const Graph &cg = levels.back();
    int64_t tot = cg.total();
    int64_t maxw[2];
    maxw[0] = maxw[1] = (int64_t)((1.0 + opt.imbalance) * 0.5 * (double)tot) + 1;
    std::vector<int> best;
    int64_t best_cut = -1;
    for (int t = 0; t < opt.init_tries; t++) {
        std::vector<int> p;
        grow_bisection(cg, rng, tot / 2, p);
        fm_refine(cg, p, maxw, opt.fm_passes);
        int64_t c = cut_of(cg, p);
        if (best_cut < 0 || c < best_cut) { best_cut = c; best = p; }
    }
    part = best;
    for (int l = (int)levels.size() - 2; l >= 0; l--) {
        const Graph &fg = levels[l];
        std::vector<int> fp(fg.n);
        for (int v = 0; v < fg.n; v++) fp[v] = part[maps[l][v]];
        int64_t ft = fg.total();
        maxw[0] = maxw[1] = (int64_t)((1.0 + opt.imbalance) * 0.5 * (double)ft) + 1;
        fm_refine(fg, fp, maxw, opt.fm_passes);
        part.swap(fp);
    }
}

// minimum vertex cover of the cut edges (Hopcroft-Karp + Koenig); marks the
// cover as part 2
void edge_to_vertex_separator(const Graph &g, std::vector<int> &part) {
    int n = g.n;
    std::vector<int> lid(n, -1), rid(n, -1), lv, rv;
    for (int v = 0; v < n; v++) {
        bool bnd = false;
        for (int e = g.xadj[v]; e < g.xadj[v + 1] && !bnd; e++) bnd = part[g.adj[e]] != part[v];
        if (!bnd) continue;
        if (part[v] == 0) { lid[v] = (int)lv.size(); lv.push_back(v); }
        else { rid[v] = (int)rv.size(); rv.push_back(v); }
    }
    int nl = (int)lv.size(), nr = (int)rv.size();
    std::vector<int> bx(nl + 1, 0), badj;
    for (int i = 0; i < nl; i++) {
        int v = lv[i];
        for (int e = g.xadj[v]; e < g.xadj[v + 1]; e++)
            if (part[g.adj[e]] == 1) badj.push_back(rid[g.adj[e]]);
        bx[i + 1] = (int)badj.size();
    }
    std::vector<int> ml(nl, -1), mr(nr, -1), dist(nl), it(nl);
    const int INF = 1 << 30;
    while (true) {
        std::queue<int> q;
        bool found = false;
        for (int i = 0; i < nl; i++) {
            if (ml[i] < 0) { dist[i] = 0; q.push(i); }
            else dist[i] = INF;
        }
        while (!q.empty()) {
            int i = q.front(); q.pop();
            for (int e = bx[i]; e < bx[i + 1]; e++) {
                int j = mr[badj[e]];
                if (j < 0) found = true;
                else if (dist[j] == INF) { dist[j] = dist[i] + 1; q.push(j); }
            }
        }
        if (!found) break;
        // iterative DFS along the BFS layers
        for (int i = 0; i < nl; i++) it[i] = bx[i];
        for (int s = 0; s < nl; s++) {
            if (ml[s] >= 0) continue;
            std::vector<int> stk{s};
            bool aug = false;
            while (!stk.empty() && !aug) {
                int i = stk.back();
                if (it[i] == bx[i + 1]) { dist[i] = INF; stk.pop_back(); continue; }
                int r = badj[it[i]];
                int j = mr[r];
                if (j < 0) {
                    // augment along the stack
                    for (int k = (int)stk.size() - 1; k >= 0; k--) {
                        int li = stk[k];
                        int rr = badj[it[li]];
                        int prev = ml[li];
                        ml[li] = rr;
                        mr[rr] = li;
                        (void)prev;
                    }
                    aug = true;
                } else if (dist[j] == dist[i] + 1) {
                    stk.push_back(j);
                } else {
                    it[i]++;
                }
            }
        }
    }
    // Koenig: Z = vertices reachable from free left vertices by alternating paths
    std::vector<char> zl(nl, 0), zr(nr, 0);
    std::queue<int> q;
    for (int i = 0; i < nl; i++) if (ml[i] < 0) { zl[i] = 1; q.push(i); }
    while (!q.empty()) {
        int i = q.front(); q.pop();
        for (int e = bx[i]; e < bx[i + 1]; e++) {
            int r = badj[e];
            if (zr[r] || ml[i] == r) continue;
            zr[r] = 1;
            int j = mr[r];
            if (j >= 0 && !zl[j]) { zl[j] = 1; q.push(j); }
        }
    }
    for (int i = 0; i < nl; i++) if (!zl[i]) part[lv[i]] = 2;
    for (int r = 0; r < nr; r++) if (zr[r]) part[rv[r]] = 2;
}

struct NdBuilder {
    const NdOptions &opt;
    Rng rng;
    std::vector<int32_t> order;        // emission order of old indices (new -> old)
    std::vector<Front> fronts;
    explicit NdBuilder(const NdOptions &o) : opt(o), rng(o.seed) {}

    int leaf(const std::vector<int> &glob) {
        Front f;
        f.first = (int32_t)order.size();
        f.p = (int32_t)glob.size();
        for (int v : glob) order.push_back(v);
        fronts.push_back(f);
        return (int)fronts.size() - 1;
    }

    // g: subgraph, glob: subgraph vertex -> original index
    int dissect(const Graph &g, const std::vector<int> &glob) {
        if (g.n <= opt.leaf_size) return leaf(glob);
        std::vector<int> part;
        multilevel_bisect(g, opt, rng, part);
        edge_to_vertex_separator(g, part);
        int64_t n0 = 0, n1 = 0;
        for (int v = 0; v < g.n; v++) { n0 += part[v] == 0; n1 += part[v] == 1; }
        if (n0 == 0 || n1 == 0) return leaf(glob);
        std::vector<int> children;
        for (int side = 0; side < 2; side++) {
            std::vector<int> sub2g;
            Graph s = induced(g, part, side, sub2g);
            std::vector<int> sg(sub2g.size());
            for (size_t i = 0; i < sub2g.size(); i++) sg[i] = glob[sub2g[i]];
            children.push_back(dissect(s, sg));
        }
        Front f;
        f.first = (int32_t)order.size();
        for (int v = 0; v < g.n; v++)
            if (part[v] == 2) order.push_back(glob[v]);
        f.p = (int32_t)order.size() - f.first;
        f.children = children;
        fronts.push_back(f);
        int id = (int)fronts.size() - 1;
        for (int c : children) fronts[c].parent = id;
        return id;
    }
};

}  // namespace

FrontTree build_front_tree(const Pattern &A, const NdOptions &opt) {
    auto t0 = std::chrono::steady_clock::now();
    FrontTree t;
    t.n = A.n;
    Graph g;
    g.n = (int)A.n;
    g.xadj.assign(g.n + 1, 0);
    g.vw.assign(g.n, 1);
    for (int v = 0; v < g.n; v++) {
        for (int e = A.rowptr[v]; e < A.rowptr[v + 1]; e++) {
            int u = A.col[e];
            if (u == v) continue;
            g.adj.push_back(u);
            g.ew.push_back(1);
        }
        g.xadj[v + 1] = (int)g.adj.size();
    }
    NdBuilder b(opt);
    std::vector<int> glob(g.n);
    std::iota(glob.begin(), glob.end(), 0);
    b.dissect(g, glob);
    if ((int64_t)b.order.size() != A.n) throw std::logic_error("nested dissection lost vertices");
    t.perm = b.order;
    t.iperm.assign(A.n, -1);
    for (int64_t k = 0; k < A.n; k++) t.iperm[t.perm[k]] = (int32_t)k;
    t.fronts = std::move(b.fronts);

    // contribution rows, bottom-up (fronts are in post-order)
    std::vector<std::vector<int32_t>> cr(t.fronts.size());
    for (size_t fi = 0; fi < t.fronts.size(); fi++) {
        Front &f = t.fronts[fi];
        int32_t end = f.first + f.p;
        std::vector<int32_t> rows;
        for (int32_t j = f.first; j < end; j++) {
            int32_t old = t.perm[j];
            for (int32_t e = A.rowptr[old]; e < A.rowptr[old + 1]; e++) {
                int32_t i = t.iperm[A.col[e]];
                if (i >= end) rows.push_back(i);
            }
        }
        for (int ch : f.children)
            for (int32_t x : cr[ch])
                if (x >= end) rows.push_back(x);
        std::sort(rows.begin(), rows.end());
        rows.erase(std::unique(rows.begin(), rows.end()), rows.end());
        cr[fi] = std::move(rows);
        for (int ch : f.children) { std::vector<int32_t>().swap(cr[ch]); }
        f.c = (int32_t)cr[fi].size();
        f.cptr = (int64_t)t.contrib.size();
        t.contrib.insert(t.contrib.end(), cr[fi].begin(), cr[fi].end());
        int lvl = 0;
        for (int ch : f.children) lvl = std::max(lvl, t.fronts[ch].level + 1);
        f.level = lvl;
        t.n_levels = std::max(t.n_levels, lvl + 1);
        double p = f.p, c = f.c;
        t.nnz_factor += (int64_t)f.p * f.p + 2LL * f.p * f.c;
        t.front_entries += (int64_t)f.m() * f.m();
        t.flops += 2.0 / 3.0 * p * p * p + 2.0 * p * p * c + 2.0 * p * c * c;
        t.max_m = std::max<int64_t>(t.max_m, f.m());
        t.max_p = std::max<int64_t>(t.max_p, f.p);
    }
    t.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return t;
}

void child_relative_map(const FrontTree &t, int ch, std::vector<int32_t> &map) {
    const Front &c = t.fronts[ch];
    const Front &f = t.fronts[c.parent];
    const int32_t *fc = t.contrib.data() + f.cptr;
    map.resize(c.c);
    for (int32_t k = 0; k < c.c; k++) {
        int32_t x = t.contrib[c.cptr + k];
        if (x < f.first + f.p) {
            map[k] = x - f.first;
        } else {
            const int32_t *it = std::lower_bound(fc, fc + f.c, x);
            map[k] = f.p + (int32_t)(it - fc);
        }
    }
}

}  // namespace mbl
