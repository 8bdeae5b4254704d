// Recursive-bisection hypergraph partitioner for the three reorderings.
//
//  * Column-net model (Section 3.1): rows are vertices, columns are nets.
//    Cutsize under the connectivity metric, cut nets split in recursive
//    bisection, bounds Theorem 1.
//  * Enhanced row-column-net model (Section 3.2): nonzeros are vertices;
//    column nets cost 1 and are split when cut (connectivity metric); a row
//    net costs nnz(r_i) and, when cut, is removed together with its vertices
//    (cut-net metric), which sends row i to the row border R_B.  Bound:
//    Theorem 2.
//  * Row-column-net model (Section 4.1): nonzeros are vertices, rows and
//    columns are nets under the connectivity metric.  Bound: Corollary 4,
//    which weighs rows and columns alike (cost 1 each); the split weighs a
//    row net kSplitRowNetCostDefault times a column net unless the caller
//    gives another cost (see row_column_net).
//
// Each bisection is multilevel: matching-based coarsening that favours
// vertices sharing many small nets (heavy connectivity), greedy growing
// initial bisections on the coarsest hypergraph, and boundary
// Fiduccia-Mattheyses refinement while projecting back.  The recursion stops
// at K parts; with a window budget it continues inside every part until each
// leaf's vector window fits (the paper recurses until a part fits the cache,
// Section 5.1).  Everything is seeded; subtrees may run on different threads
// without changing the result.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <future>
#include <mutex>
#include <numeric>
#include <thread>

#include "spx_internal.h"

namespace spx {

namespace {

std::atomic<int32_t> g_threads{0};

struct Rng {
    uint64_t s;
    explicit Rng(uint64_t seed) : s(seed ^ 0x9E3779B97F4A7C15ull) {}
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    uint32_t below(uint32_t n) { return n ? (uint32_t)(next() % n) : 0; }
};

uint64_t mix(uint64_t a, uint64_t b) {
    Rng r(a * 0x100000001B3ull + b);
    return r.next();
}

constexpr int32_t kCoarsenTo = 320;
constexpr int64_t kMatchNetCap = 32;    // nets larger than this are ignored by clustering
constexpr int64_t kCoarseNetCap = 512;  // nets larger than this are left out of coarse levels
constexpr int kInitTrials = 8;
constexpr int32_t kAbsorbFrom = 20000;  // first-level absorption above this many vertices

// ------------------------------------------------------------ indexed heap
class MaxHeap {
  public:
    void init(int32_t n) {
        pos_.assign(n, -1);
        key_.assign(n, 0);
        heap_.clear();
    }
    bool contains(int32_t v) const { return pos_[v] >= 0; }
    bool empty() const { return heap_.empty(); }
    int32_t top() const { return heap_[0]; }
    int64_t key(int32_t v) const { return key_[v]; }
    void push(int32_t v, int64_t k) {
        key_[v] = k;
        pos_[v] = (int32_t)heap_.size();
        heap_.push_back(v);
        up(pos_[v]);
    }
    void update(int32_t v, int64_t k) {
        int64_t old = key_[v];
        key_[v] = k;
        if (k > old) up(pos_[v]);
        else down(pos_[v]);
    }
    void erase(int32_t v) {
        int32_t i = pos_[v];
        int32_t last = heap_.back();
        heap_.pop_back();
        pos_[v] = -1;
        if (last != v) {
            heap_[i] = last;
            pos_[last] = i;
            up(i);
            down(pos_[last]);
        }
    }
    // heapify after bulk insertion
    void bulk(const std::vector<int32_t> &vs, const std::vector<int64_t> &keys) {
        heap_ = vs;
        for (size_t i = 0; i < heap_.size(); ++i) {
            key_[heap_[i]] = keys[heap_[i]];
            pos_[heap_[i]] = (int32_t)i;
        }
        for (int32_t i = (int32_t)heap_.size() / 2 - 1; i >= 0; --i) down(i);
    }

  private:
    bool less(int32_t a, int32_t b) const {  // a below b in the heap
        return key_[a] < key_[b] || (key_[a] == key_[b] && a > b);
    }
    void up(int32_t i) {
        while (i > 0) {
            int32_t p = (i - 1) / 2;
            if (!less(heap_[p], heap_[i])) break;
            swap(i, p);
            i = p;
        }
    }
    void down(int32_t i) {
        int32_t n = (int32_t)heap_.size();
        for (;;) {
            int32_t l = 2 * i + 1, r = l + 1, b = i;
            if (l < n && less(heap_[b], heap_[l])) b = l;
            if (r < n && less(heap_[b], heap_[r])) b = r;
            if (b == i) break;
            swap(i, b);
            i = b;
        }
    }
    void swap(int32_t i, int32_t j) {
        std::swap(heap_[i], heap_[j]);
        pos_[heap_[i]] = i;
        pos_[heap_[j]] = j;
    }
    std::vector<int32_t> heap_, pos_;
    std::vector<int64_t> key_;
};

// --------------------------------------------------------- 2-way state + FM
struct Bipart {
    const Hypergraph &H;
    std::vector<uint8_t> &side;
    std::vector<int32_t> cnt[2];
    std::vector<int64_t> gain;
    std::vector<uint8_t> locked;
    int64_t W[2] = {0, 0};
    int64_t maxW[2] = {0, 0};
    int64_t cut = 0;
    MaxHeap heap[2];

    Bipart(const Hypergraph &h, std::vector<uint8_t> &s) : H(h), side(s) {}

    void set_balance(double frac0, double eps) {
        int64_t tot = H.total_weight();
        int64_t maxv = 0;
        for (int32_t v = 0; v < H.nv; ++v) maxv = std::max(maxv, H.vw[v]);
        double t0 = frac0 * (double)tot, t1 = (1.0 - frac0) * (double)tot;
        maxW[0] = std::max<int64_t>((int64_t)(t0 * (1.0 + eps)), (int64_t)t0 + maxv);
        maxW[1] = std::max<int64_t>((int64_t)(t1 * (1.0 + eps)), (int64_t)t1 + maxv);
    }

    void recount() {
        cnt[0].assign(H.nn, 0);
        cnt[1].assign(H.nn, 0);
        W[0] = W[1] = 0;
        for (int32_t v = 0; v < H.nv; ++v) W[side[v]] += H.vw[v];
        cut = 0;
        for (int32_t n = 0; n < H.nn; ++n) {
            int32_t c0 = 0, c1 = 0;
            for (int64_t p = H.xpins[n]; p < H.xpins[n + 1]; ++p) (side[H.pins[p]] ? c1 : c0)++;
            cnt[0][n] = c0;
            cnt[1][n] = c1;
            if (c0 && c1) cut += H.nc[n];
        }
    }

    int64_t vgain(int32_t v) const {
        int s = side[v];
        int64_t g = 0;
        for (int64_t q = H.xnets[v]; q < H.xnets[v + 1]; ++q) {
            int32_t n = H.vnets[q];
            if (cnt[s][n] == 1) g += H.nc[n];
            if (cnt[1 - s][n] == 0) g -= H.nc[n];
        }
        return g;
    }

    void compute_gains() {
        gain.resize(H.nv);
        for (int32_t v = 0; v < H.nv; ++v) gain[v] = vgain(v);
    }

    void touch(int32_t u, int64_t delta) {
        gain[u] += delta;
        if (locked[u]) return;
        MaxHeap &h = heap[side[u]];
        if (h.contains(u)) h.update(u, gain[u]);
        else h.push(u, gain[u]);
    }

    // Move v to the other side, updating counts and the gains of free pins
    // (Fiduccia-Mattheyses rules for the cut-net metric of a bisection).
    void move(int32_t v) {
        int F = side[v], T = 1 - F;
        cut -= gain[v];
        for (int64_t q = H.xnets[v]; q < H.xnets[v + 1]; ++q) {
            int32_t n = H.vnets[q];
            int64_t c = H.nc[n];
            int32_t tT = cnt[T][n];
            if (tT == 0) {
                for (int64_t p = H.xpins[n]; p < H.xpins[n + 1]; ++p) {
                    int32_t u = H.pins[p];
                    if (u != v) touch(u, c);
                }
            } else if (tT == 1) {
                for (int64_t p = H.xpins[n]; p < H.xpins[n + 1]; ++p) {
                    int32_t u = H.pins[p];
                    if (u != v && side[u] == T) { touch(u, -c); break; }
                }
            }
            cnt[F][n]--;
            cnt[T][n]++;
            int32_t nF = cnt[F][n];
            if (nF == 0) {
                for (int64_t p = H.xpins[n]; p < H.xpins[n + 1]; ++p) {
                    int32_t u = H.pins[p];
                    if (u != v) touch(u, -c);
                }
            } else if (nF == 1) {
                for (int64_t p = H.xpins[n]; p < H.xpins[n + 1]; ++p) {
                    int32_t u = H.pins[p];
                    if (u != v && side[u] == F) { touch(u, c); break; }
                }
            }
        }
        side[v] = (uint8_t)T;
        W[F] -= H.vw[v];
        W[T] += H.vw[v];
        gain[v] = -gain[v];
    }

    bool balanced() const { return W[0] <= maxW[0] && W[1] <= maxW[1]; }
    int64_t imbalance() const {
        return std::max<int64_t>(0, W[0] - maxW[0]) + std::max<int64_t>(0, W[1] - maxW[1]);
    }

    // One FM pass with rollback to the best prefix.  Returns true if the
    // cut (or the balance) improved.
    bool fm_pass(int64_t max_bad) {
        locked.assign(H.nv, 0);
        heap[0].init(H.nv);
        heap[1].init(H.nv);
        std::vector<int32_t> b0, b1;
        for (int32_t v = 0; v < H.nv; ++v) {
            bool boundary = false;
            for (int64_t q = H.xnets[v]; q < H.xnets[v + 1] && !boundary; ++q) {
                int32_t n = H.vnets[q];
                boundary = cnt[0][n] > 0 && cnt[1][n] > 0;
            }
            if (boundary || !balanced()) (side[v] ? b1 : b0).push_back(v);
        }
        heap[0].bulk(b0, gain);
        heap[1].bulk(b1, gain);
        std::vector<int32_t> moves;
        int64_t start_cut = cut, start_imb = imbalance();
        int64_t best_cut = cut, best_imb = start_imb;
        size_t best_len = 0;
        int64_t bad = 0;
        while (bad < max_bad) {
            int pick = -1;
            int64_t bestg = INT64_MIN;
            for (int s = 0; s < 2; ++s) {
                if (heap[s].empty()) continue;
                int32_t v = heap[s].top();
                int T = 1 - s;
                bool over = W[s] > maxW[s];
                bool fits = W[T] + H.vw[v] <= maxW[T];
                if (!fits && !over) continue;
                int64_t g = heap[s].key(v) + (over ? (int64_t)1 << 40 : 0);
                if (g > bestg) { bestg = g; pick = s; }
            }
            if (pick < 0) break;
            int32_t v = heap[pick].top();
            heap[pick].erase(v);
            locked[v] = 1;
            move(v);
            moves.push_back(v);
            int64_t imb = imbalance();
            if (imb < best_imb || (imb == best_imb && cut < best_cut)) {
                best_imb = imb;
                best_cut = cut;
                best_len = moves.size();
                bad = 0;
            } else {
                ++bad;
            }
        }
        for (size_t i = moves.size(); i > best_len; --i) {
            int32_t v = moves[i - 1];
            locked[v] = 0;
            move(v);
        }
        return best_imb < start_imb || best_cut < start_cut;
    }

    void refine(int passes, int64_t max_bad) {
        for (int p = 0; p < passes; ++p)
            if (!fm_pass(max_bad)) break;
    }
};

// Greedy hypergraph growing from a random seed vertex, then FM.
int64_t initial_bisection(const Hypergraph &H, double frac0, double eps, Rng &rng,
                          std::vector<uint8_t> &best_side) {
    int64_t best = INT64_MAX, best_imb = INT64_MAX;
    std::vector<uint8_t> side(H.nv);
    int64_t tot = H.total_weight();
    // effort scaled to the coarse hypergraph: a few trials when it is large
    int trials = H.pins.size() > 4000000 ? 2 : (H.pins.size() > 1000000 ? 4 : kInitTrials);
    for (int t = 0; t < trials; ++t) {
        std::fill(side.begin(), side.end(), 1);
        Bipart B(H, side);
        B.set_balance(frac0, eps);
        B.recount();
        B.compute_gains();
        B.locked.assign(H.nv, 0);
        B.heap[0].init(H.nv);
        B.heap[1].init(H.nv);
        int64_t target0 = (int64_t)(frac0 * (double)tot);
        if (t % 4 == 3) {
            // random assignment trial
            for (int32_t v = 0; v < H.nv; ++v)
                if (B.W[0] < target0 && rng.below(1000) < (uint32_t)(frac0 * 1000)) {
                    B.side[v] = 0;
                    B.W[0] += H.vw[v];
                    B.W[1] -= H.vw[v];
                }
            B.recount();
            B.compute_gains();
        } else {
            std::vector<int32_t> all(H.nv);
            std::iota(all.begin(), all.end(), 0);
            B.heap[1].bulk(all, B.gain);
            int32_t seed_v = (int32_t)rng.below((uint32_t)H.nv);
            // raise the seed vertex to the top
            B.heap[1].update(seed_v, (int64_t)1 << 50);
            while (B.W[0] < target0 && !B.heap[1].empty()) {
                int32_t v = B.heap[1].top();
                B.heap[1].erase(v);
                B.locked[v] = 1;
                B.move(v);
            }
            B.recount();
            B.compute_gains();
        }
        B.refine(3, std::max<int64_t>(50, std::min<int64_t>(H.nv / 4, 400)));
        int64_t imb = B.imbalance();
        if (imb < best_imb || (imb == best_imb && B.cut < best)) {
            best = B.cut;
            best_imb = imb;
            best_side = side;
        }
    }
    return best;
}

// Heavy-connectivity clustering: vertices are visited in random order and an
// unclustered vertex joins the neighbouring cluster (or pairs with the
// unclustered neighbour) it shares the most net weight with, each shared net
// n contributing cost(n) / (|n| - 1); nets above kMatchNetCap pins are
// ignored.  Cluster weights are capped at maxw.
void match_hcc(const Hypergraph &H, int64_t maxw, Rng &rng, std::vector<int32_t> &cmap,
               int32_t &ncoarse) {
    int32_t nv = H.nv;
    std::vector<int32_t> order(nv);
    std::iota(order.begin(), order.end(), 0);
    for (int32_t i = nv - 1; i > 0; --i) std::swap(order[i], order[rng.below((uint32_t)i + 1)]);
    std::vector<int32_t> cl(nv, -1);
    std::vector<int64_t> cw;  // cluster weights
    std::vector<float> vscore(nv, 0.f), cscore;
    std::vector<int32_t> vt, ct;
    int64_t dbg_none = 0, dbg_small = 0, dbg_blocked = 0;
    cscore.reserve(nv / 2 + 1);
    for (int32_t v : order) {
        if (cl[v] >= 0) continue;
        vt.clear();
        ct.clear();
        for (int64_t q = H.xnets[v]; q < H.xnets[v + 1]; ++q) {
            int32_t n = H.vnets[q];
            int64_t sz = H.xpins[n + 1] - H.xpins[n];
            if (sz < 2 || sz > kMatchNetCap) continue;
            ++dbg_small;
            float w = (float)H.nc[n] / (float)(sz - 1);
            for (int64_t p = H.xpins[n]; p < H.xpins[n + 1]; ++p) {
                int32_t u = H.pins[p];
                if (u == v) continue;
                int32_t c = cl[u];
                if (c >= 0) {
                    if (cw[c] + H.vw[v] > maxw) { ++dbg_blocked; continue; }
                    if (cscore[c] == 0.f) ct.push_back(c);
                    cscore[c] += w;
                } else {
                    if (H.vw[u] + H.vw[v] > maxw) continue;
                    if (vscore[u] == 0.f) vt.push_back(u);
                    vscore[u] += w;
                }
            }
        }
        if (vt.empty() && ct.empty()) {
            // only large nets: look at a bounded prefix of each of them
            ++dbg_none;
            for (int64_t q = H.xnets[v]; q < H.xnets[v + 1]; ++q) {
                int32_t n = H.vnets[q];
                int64_t sz = H.xpins[n + 1] - H.xpins[n];
                if (sz <= kMatchNetCap) continue;
                float w = (float)H.nc[n] / (float)(sz - 1);
                int64_t end = std::min(H.xpins[n + 1], H.xpins[n] + kMatchNetCap);
                for (int64_t p = H.xpins[n]; p < end; ++p) {
                    int32_t u = H.pins[p];
                    if (u == v) continue;
                    int32_t c = cl[u];
                    if (c >= 0) {
                        if (cw[c] + H.vw[v] > maxw) continue;
                        if (cscore[c] == 0.f) ct.push_back(c);
                        cscore[c] += w;
                    } else {
                        if (H.vw[u] + H.vw[v] > maxw) continue;
                        if (vscore[u] == 0.f) vt.push_back(u);
                        vscore[u] += w;
                    }
                }
            }
        }
        int32_t bu = -1, bc = -1;
        float bs = 0.f;
        // rating = shared net weight per unit of merged weight, which keeps
        // clusters of similar size
        for (int32_t u : vt) {
            float r = vscore[u] / (float)(H.vw[u] + H.vw[v]);
            if (r > bs) { bs = r; bu = u; bc = -1; }
            vscore[u] = 0.f;
        }
        for (int32_t c : ct) {
            float r = cscore[c] / (float)(cw[c] + H.vw[v]);
            if (r > bs) { bs = r; bc = c; bu = -1; }
            cscore[c] = 0.f;
        }
        if (bc >= 0) {
            cl[v] = bc;
            cw[bc] += H.vw[v];
        } else {
            int32_t c = (int32_t)cw.size();
            cw.push_back(H.vw[v]);
            cscore.push_back(0.f);
            cl[v] = c;
            if (bu >= 0) {
                cl[bu] = c;
                cw[c] += H.vw[bu];
            }
        }
    }
    if (getenv("SPX_DEBUG") && nv > 50000)
        fprintf(stderr, "    hcc nv=%d none=%lld smallnets=%lld blocked=%lld clusters=%zu\n", nv,
                (long long)dbg_none, (long long)dbg_small, (long long)dbg_blocked, cw.size());
    // renumber clusters by first vertex so the result does not depend on
    // the visiting order beyond the clustering itself
    std::vector<int32_t> ren(cw.size(), -1);
    cmap.assign(nv, -1);
    ncoarse = 0;
    for (int32_t v = 0; v < nv; ++v) {
        int32_t c = cl[v];
        if (ren[c] < 0) ren[c] = ncoarse++;
        cmap[v] = ren[c];
    }
}

// Absorption clustering over nets, for the first level of large
// hypergraphs: nets are visited from the smallest up and each net gathers its
// still unclustered pins into clusters of at most maxw weight; a lone
// unclustered pin joins the cluster of the net's first clustered pin when the
// weight allows.  One pass over the pins, mostly sequential in memory.
void absorb_nets(const Hypergraph &H, int64_t maxw, int64_t heavy_maxw, std::vector<int32_t> &cmap,
                 int32_t &ncoarse) {
    int32_t nv = H.nv;
    // strongest connections first: cost / (|n| - 1) descending, then size
    std::vector<std::pair<double, int32_t>> rated;
    for (int32_t n = 0; n < H.nn; ++n) {
        int64_t sz = H.xpins[n + 1] - H.xpins[n];
        if (sz >= 2 && (sz <= kMatchNetCap || H.nc[n] >= sz - 1))
            rated.emplace_back(-(double)H.nc[n] / (double)(sz - 1) + 1e-9 * (double)sz, n);
    }
    std::stable_sort(rated.begin(), rated.end(),
                     [](const std::pair<double, int32_t> &a, const std::pair<double, int32_t> &b) {
                         return a.first < b.first;
                     });
    std::vector<int32_t> order(rated.size());
    for (size_t i = 0; i < rated.size(); ++i) order[i] = rated[i].second;
    rated.clear();
    rated.shrink_to_fit();
    std::vector<int32_t> cl(nv, -1);
    std::vector<int64_t> cw;
    std::vector<int32_t> fresh;
    for (int32_t n : order) {
        fresh.clear();
        int32_t host = -1;
        // a net at least as strong as a two-pin net (cost >= |n| - 1, the row
        // nets of the enhanced model) is kept together
        int64_t sz = H.xpins[n + 1] - H.xpins[n];
        int64_t cap = H.nc[n] >= sz - 1 && sz > 2 ? heavy_maxw : maxw;
        for (int64_t p = H.xpins[n]; p < H.xpins[n + 1]; ++p) {
            int32_t u = H.pins[p];
            if (cl[u] < 0) fresh.push_back(u);
            else if (host < 0) host = cl[u];
        }
        if (fresh.empty()) continue;
        if (fresh.size() == 1) {
            int32_t u = fresh[0];
            if (host >= 0 && cw[host] + H.vw[u] <= cap) {
                cl[u] = host;
                cw[host] += H.vw[u];
            }
            continue;
        }
        int32_t c = -1;
        for (int32_t u : fresh) {
            if (c < 0 || cw[c] + H.vw[u] > cap) {
                c = (int32_t)cw.size();
                cw.push_back(0);
            }
            cl[u] = c;
            cw[c] += H.vw[u];
        }
    }
    if (getenv("SPX_DEBUG")) {
        int64_t heavy = 0, single = 0;
        for (int32_t n : order) {
            int64_t sz = H.xpins[n + 1] - H.xpins[n];
            if (H.nc[n] >= sz - 1 && sz > 2) ++heavy;
        }
        for (int32_t v = 0; v < nv; ++v) single += cl[v] < 0;
        fprintf(stderr, "    absorb nv=%d nets=%zu heavy=%lld clusters=%zu singletons=%lld maxw=%lld heavyw=%lld\n", nv,
                order.size(), (long long)heavy, cw.size(), (long long)single, (long long)maxw, (long long)heavy_maxw);
    }
    std::vector<int32_t> ren(cw.size(), -1);
    cmap.assign(nv, -1);
    ncoarse = 0;
    for (int32_t v = 0; v < nv; ++v) {
        if (cl[v] < 0) { cmap[v] = ncoarse++; continue; }
        if (ren[cl[v]] < 0) ren[cl[v]] = ncoarse++;
        cmap[v] = ren[cl[v]];
    }
}

// The nets [n0, n1) of H as clusters: each net's distinct clusters in
// ascending order with their hash, or nothing when fewer than two or more
// than kCoarseNetCap remain.  A net's result depends on that net alone.
struct ReducedNets {
    std::vector<int64_t> off;  // net n0 + i holds pins[off[i], off[i + 1])
    std::vector<int32_t> pins;
    std::vector<uint64_t> hash;
};

void reduce_nets(const Hypergraph &H, const std::vector<int32_t> &cmap, int32_t nc, int32_t n0, int32_t n1,
                 ReducedNets &R) {
    std::vector<int32_t> mark(nc, -1);
    std::vector<int32_t> buf;
    R.off.assign((size_t)(n1 - n0) + 1, 0);
    R.hash.assign((size_t)(n1 - n0), 0);
    R.pins.clear();
    for (int32_t n = n0; n < n1; ++n) {
        buf.clear();
        for (int64_t p = H.xpins[n]; p < H.xpins[n + 1]; ++p) {
            int32_t c = cmap[H.pins[p]];
            if (mark[c] != n) { mark[c] = n; buf.push_back(c); }
        }
        if (buf.size() >= 2 && (int64_t)buf.size() <= kCoarseNetCap) {
            std::sort(buf.begin(), buf.end());
            uint64_t h = 1469598103934665603ull ^ buf.size();
            for (int32_t c : buf) h = (h ^ (uint64_t)c) * 1099511628211ull;
            h ^= H.nrow.empty() ? 0 : H.nrow[n];
            R.hash[n - n0] = h;
            R.pins.insert(R.pins.end(), buf.begin(), buf.end());
        }
        R.off[n - n0 + 1] = (int64_t)R.pins.size();
    }
}

// Contract clusters into a coarse hypergraph.  Nets reduced to one cluster
// vanish, nets spanning more than kCoarseNetCap clusters are left out of the
// coarse levels (they are cut by nearly every bisection and only slow the
// coarse search down; the finest level keeps them), and nets with identical
// pin sets are merged by adding their costs.  Large hypergraphs reduce their
// nets on up to `threads` threads; the merge then walks the nets in order, so
// the result does not depend on the thread count.
void contract(const Hypergraph &H, const std::vector<int32_t> &cmap, int32_t nc, Hypergraph &C,
              int32_t threads) {
    C.nv = nc;
    C.vw.assign(nc, 0);
    for (int32_t v = 0; v < H.nv; ++v) C.vw[cmap[v]] += H.vw[v];
    // one thread per 2^20 pins, at most `threads`
    int32_t T = (int32_t)std::min<size_t>(H.pins.size() >> 20, (size_t)std::max<int32_t>(1, threads));
    T = std::max<int32_t>(1, std::min<int32_t>(T, H.nn));
    // chunks of nets holding about equal numbers of pins
    std::vector<int32_t> cut(T + 1, H.nn);
    cut[0] = 0;
    for (int32_t t = 1; t < T; ++t) {
        int64_t want = (int64_t)((double)H.pins.size() * t / T);
        cut[t] = (int32_t)(std::lower_bound(H.xpins.begin(), H.xpins.begin() + H.nn, want) - H.xpins.begin());
        cut[t] = std::max(cut[t], cut[t - 1]);
    }
    std::vector<ReducedNets> R(T);
    if (T == 1) {
        reduce_nets(H, cmap, nc, 0, H.nn, R[0]);
    } else {
        std::vector<std::thread> th;
        for (int32_t t = 0; t < T; ++t)
            th.emplace_back([&, t] { reduce_nets(H, cmap, nc, cut[t], cut[t + 1], R[t]); });
        for (auto &x : th) x.join();
    }
    C.xpins.clear();
    C.pins.clear();
    C.nc.clear();
    C.nrow.clear();
    C.xpins.push_back(0);
    // open-addressing table of net hashes -> coarse net id
    size_t cap = 1;
    while (cap < 2 * (size_t)H.nn + 16) cap <<= 1;
    std::vector<int32_t> table(cap, -1);
    std::vector<uint64_t> nhash;
    for (int32_t t = 0; t < T; ++t) {
        const ReducedNets &Q = R[t];
        for (int32_t n = cut[t]; n < cut[t + 1]; ++n) {
            size_t i = (size_t)(n - cut[t]);
            int64_t len = Q.off[i + 1] - Q.off[i];
            if (len == 0) continue;
            const int32_t *b = Q.pins.data() + Q.off[i];
            uint64_t h = Q.hash[i];
            uint8_t row = H.nrow.empty() ? 0 : H.nrow[n];
            size_t slot = (size_t)(h ^ (h >> 29)) & (cap - 1);
            int32_t found = -1;
            while (table[slot] >= 0) {
                int32_t e = table[slot];
                if (nhash[e] == h && C.nrow[e] == row && C.xpins[e + 1] - C.xpins[e] == len &&
                    std::equal(b, b + len, C.pins.begin() + C.xpins[e])) {
                    found = e;
                    break;
                }
                slot = (slot + 1) & (cap - 1);
            }
            if (found >= 0) {
                C.nc[found] += H.nc[n];
                continue;
            }
            table[slot] = (int32_t)C.nc.size();
            nhash.push_back(h);
            C.pins.insert(C.pins.end(), b, b + len);
            C.xpins.push_back((int64_t)C.pins.size());
            C.nc.push_back(H.nc[n]);
            C.nrow.push_back(row);
        }
    }
    C.nn = (int32_t)C.nc.size();
    C.build_vertex_side();
}

}  // namespace

int32_t num_threads() {
    int32_t t = g_threads.load();
    if (t <= 0) {
        unsigned hc = std::thread::hardware_concurrency();
        t = (int32_t)std::max(1u, std::min(hc, 16u));
    }
    return t;
}
void set_num_threads(int32_t t) { g_threads.store(t); }

int64_t Hypergraph::total_weight() const {
    int64_t s = 0;
    for (int64_t w : vw) s += w;
    return s;
}

void Hypergraph::build_vertex_side() {
    xnets.assign((size_t)nv + 1, 0);
    for (int32_t u : pins) xnets[u + 1]++;
    for (int32_t v = 0; v < nv; ++v) xnets[v + 1] += xnets[v];
    vnets.assign(pins.size(), 0);
    std::vector<int64_t> fill(xnets.begin(), xnets.end() - 1);
    for (int32_t n = 0; n < nn; ++n)
        for (int64_t p = xpins[n]; p < xpins[n + 1]; ++p) vnets[fill[pins[p]]++] = n;
}

static bool debug_on() {
    static int on = -1;
    if (on < 0) on = getenv("SPX_DEBUG") ? 1 : 0;
    return on == 1;
}

static double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

int64_t bisect(const Hypergraph &H, double frac0, double eps, uint64_t seed,
               std::vector<uint8_t> &side, int32_t threads) {
    side.assign(H.nv, 0);
    if (H.nv <= 1) return 0;
    double tb = now_s(), tm = 0, tc = 0, tf = 0;
    Rng rng(seed);
    std::vector<std::unique_ptr<Hypergraph>> levels;
    std::vector<std::vector<int32_t>> maps;
    const Hypergraph *cur = &H;
    int64_t tot = H.total_weight();
    int64_t maxv = 0;
    for (int64_t w : H.vw) maxv = std::max(maxv, w);
    int64_t maxw = std::max<int64_t>(maxv, tot / (2 * kCoarsenTo) + 1);
    while (cur->nv > kCoarsenTo) {
        std::vector<int32_t> cmap;
        int32_t nc = 0;
        double t1 = now_s();
        // clusters may grow to a few times the current average vertex weight
        // absorption on the first level of very large hypergraphs, heavy
        // connectivity clustering afterwards
        if (levels.empty() && cur->nv > kAbsorbFrom) {
            int64_t aw = std::min<int64_t>(maxw, std::max<int64_t>(maxv, 8 * (tot / cur->nv) + 1));
            absorb_nets(*cur, aw, maxw, cmap, nc);
        } else {
            match_hcc(*cur, maxw, rng, cmap, nc);
        }
        tm += now_s() - t1;
        if (debug_on() && H.nv > 500000)
            fprintf(stderr, "  level nv=%d nn=%d pins=%zu -> %d (maxw %lld)\n", cur->nv, cur->nn,
                    cur->pins.size(), nc, (long long)maxw);
        if (nc > (int32_t)(0.95 * cur->nv)) break;
        auto C = std::make_unique<Hypergraph>();
        t1 = now_s();
        contract(*cur, cmap, nc, *C, threads);
        tc += now_s() - t1;
        // stop once the pins stop shrinking and the level is small enough
        // for the initial bisection: further levels only cost time
        bool stalled = (double)C->pins.size() > 0.9 * (double)cur->pins.size();
        maps.push_back(std::move(cmap));
        levels.push_back(std::move(C));
        cur = levels.back().get();
        if (stalled && cur->nv <= 8 * kCoarsenTo) break;
    }
    std::vector<uint8_t> cs;
    double ti = now_s();
    int32_t coarse_nv = cur->nv, coarse_nn = cur->nn;
    size_t coarse_pins = cur->pins.size();
    initial_bisection(*cur, frac0, eps, rng, cs);
    ti = now_s() - ti;
    for (int l = (int)levels.size() - 1; l >= 0; --l) {
        const Hypergraph &fine = (l == 0) ? H : *levels[l - 1];
        std::vector<uint8_t> fs(fine.nv);
        for (int32_t v = 0; v < fine.nv; ++v) fs[v] = cs[maps[l][v]];
        double t1 = now_s();
        Bipart B(fine, fs);
        B.set_balance(frac0, eps);
        B.recount();
        B.compute_gains();
        int64_t max_bad = std::min<int64_t>(std::max<int64_t>(64, fine.nv / 50), 4000);
        B.refine(l == 0 ? 2 : 3, max_bad);
        tf += now_s() - t1;
        cs.swap(fs);
        levels[l].reset();
    }
    if (levels.empty() && cur == &H) {
        side = cs;
    } else {
        side = cs;
    }
    Bipart F(H, side);
    F.recount();
    if (debug_on() && H.nv > 100000)
        fprintf(stderr, "bisect nv=%d nn=%d pins=%zu levels=%zu coarse=(%d,%d,%zu) match=%.2f contract=%.2f init=%.2f fm=%.2f total=%.2f cut=%lld\n",
                H.nv, H.nn, H.pins.size(), maps.size(), coarse_nv, coarse_nn, coarse_pins, tm, tc, ti, tf, now_s() - tb, (long long)F.cut);
    return F.cut;
}

// Enhanced row-column-net model: a cut row net costs nnz(r_i); moving all of
// the row's pins to the side holding most of them removes that cost and adds
// at most one column-net cut per moved pin.  Single-vertex moves cannot see
// this (the gain appears only at the last pin), so after each bisection every
// cut row is moved whole when that strictly lowers the cutsize and keeps the
// balance.  Returns the new cutsize.
static int64_t uncut_rows(const Hypergraph &H, std::vector<uint8_t> &side, double frac0, double eps,
                   int64_t cut) {
    std::vector<int32_t> cnt0(H.nn, 0), cnt1(H.nn, 0);
    int64_t W[2] = {0, 0}, tot = 0;
    for (int32_t v = 0; v < H.nv; ++v) {
        W[side[v]] += H.vw[v];
        tot += H.vw[v];
    }
    int64_t maxW[2] = {(int64_t)(frac0 * (double)tot * (1.0 + eps)),
                       (int64_t)((1.0 - frac0) * (double)tot * (1.0 + eps))};
    for (int32_t n = 0; n < H.nn; ++n)
        for (int64_t p = H.xpins[n]; p < H.xpins[n + 1]; ++p) (side[H.pins[p]] ? cnt1 : cnt0)[n]++;
    std::vector<int32_t> *cnt[2] = {&cnt0, &cnt1};
    for (int32_t r = 0; r < H.nn; ++r) {
        if (!H.nrow[r] || cnt0[r] == 0 || cnt1[r] == 0) continue;
        int s = cnt1[r] > cnt0[r] ? 1 : 0, o = 1 - s;
        int64_t dw = 0, delta = -H.nc[r];
        for (int64_t p = H.xpins[r]; p < H.xpins[r + 1]; ++p) {
            int32_t u = H.pins[p];
            if (side[u] != o) continue;
            dw += H.vw[u];
            for (int64_t q = H.xnets[u]; q < H.xnets[u + 1]; ++q) {
                int32_t c = H.vnets[q];
                if (c == r) continue;
                bool was_cut = (*cnt[0])[c] > 0 && (*cnt[1])[c] > 0;
                (*cnt[o])[c]--;
                (*cnt[s])[c]++;
                bool now_cut = (*cnt[0])[c] > 0 && (*cnt[1])[c] > 0;
                delta += (int64_t)now_cut * H.nc[c] - (int64_t)was_cut * H.nc[c];
            }
        }
        bool ok = delta < 0 && W[s] + dw <= maxW[s];
        for (int64_t p = H.xpins[r]; p < H.xpins[r + 1]; ++p) {
            int32_t u = H.pins[p];
            if (side[u] != o) continue;
            if (ok) {
                side[u] = (uint8_t)s;
            } else {
                for (int64_t q = H.xnets[u]; q < H.xnets[u + 1]; ++q) {
                    int32_t c = H.vnets[q];
                    if (c == r) continue;
                    (*cnt[s])[c]--;
                    (*cnt[o])[c]++;
                }
            }
        }
        if (ok) {
            (*cnt[s])[r] += (*cnt[o])[r];
            (*cnt[o])[r] = 0;
            W[s] += dw;
            W[o] -= dw;
            cut += delta;
        }
    }
    return cut;
}

// ------------------------------------------------- recursive bisection

namespace {

struct Sub {
    Hypergraph H;
    std::vector<int32_t> gid;  // global id of each vertex (row or nonzero)
};

struct Leaf {
    int32_t part;
    uint64_t path;  // left-aligned bit path below the part
    int32_t depth;
    std::vector<int32_t> gid;
};

struct Ctx {
    Model model;
    int32_t K;
    int64_t window;
    uint64_t seed;
    double eps;
    const CsrHost *A;
    std::mutex mu;
    std::vector<Leaf> leaves;
    std::vector<int32_t> removed;  // eRCN: nonzeros whose row went to R_B
    std::atomic<int64_t> cut{0};
    std::atomic<int32_t> active{1};  // threads working (not waiting), this one included
};

// Column-net hypergraph of a subset of rows (vertices = rows, nets = the
// columns they touch).
Sub column_net_of_rows(const CsrHost &A, const std::vector<int32_t> &rows) {
    Sub s;
    s.gid = rows;
    int32_t nv = (int32_t)rows.size();
    std::vector<std::pair<int32_t, int32_t>> pc;  // (col, local row)
    size_t tot = 0;
    for (int32_t r : rows) tot += (size_t)(A.rowptr[r + 1] - A.rowptr[r]);
    pc.reserve(tot);
    s.H.nv = nv;
    s.H.vw.resize(nv);
    for (int32_t i = 0; i < nv; ++i) {
        int32_t r = rows[i];
        s.H.vw[i] = (int64_t)(A.rowptr[r + 1] - A.rowptr[r]) + 1;
        for (int32_t p = A.rowptr[r]; p < A.rowptr[r + 1]; ++p) pc.emplace_back(A.colidx[p], i);
    }
    std::sort(pc.begin(), pc.end());
    s.H.xpins.push_back(0);
    for (size_t t = 0; t < pc.size();) {
        size_t e = t;
        while (e < pc.size() && pc[e].first == pc[t].first) ++e;
        for (size_t q = t; q < e; ++q) s.H.pins.push_back(pc[q].second);
        s.H.xpins.push_back((int64_t)s.H.pins.size());
        s.H.nc.push_back(1);
        t = e;
    }
    s.H.nn = (int32_t)s.H.nc.size();
    s.H.build_vertex_side();
    return s;
}

// Cost of a row net in the row-column-net model of the split (the caller's
// choice through spx_split_ex; spx_split uses kSplitRowNetCostDefault).
// Corollary 4 counts a cut row and a cut column alike, as each bounds a
// cache miss, which is cost 1.  On the GPU they are not alike: a row shared
// by one more part costs a zeroed y entry and an atomic add into it, while a
// column shared by one more part costs one more read of an x entry that
// usually hits L2.  Weighting a row net 32 times a column net, the split of
// the n = 10^6 irregular matrix at K = 64 with 128 KB leaves has 1.55 M row
// slots instead of 4.71 M and its product runs 1.48 times faster (1.12 times
// without leaves); weights from 16 up give about the same.

// Row-column-net hypergraph of A: vertices are nonzeros (CSR order), nets
// are the non-empty rows then the non-empty columns.  Row nets cost nnz(r)
// in the enhanced model, row_cost otherwise.
Sub row_column_net(const CsrHost &A, bool enhanced, int64_t row_cost) {
    Sub s;
    int64_t nnz = A.nnz;
    s.gid.resize(nnz);
    std::iota(s.gid.begin(), s.gid.end(), 0);
    s.H.nv = (int32_t)nnz;
    s.H.vw.assign(nnz, 1);
    s.H.xpins.push_back(0);
    for (int32_t i = 0; i < A.m; ++i) {
        int32_t d = A.rowptr[i + 1] - A.rowptr[i];
        if (d == 0) continue;
        for (int32_t p = A.rowptr[i]; p < A.rowptr[i + 1]; ++p) s.H.pins.push_back(p);
        s.H.xpins.push_back((int64_t)s.H.pins.size());
        s.H.nc.push_back(enhanced ? d : row_cost);
        s.H.nrow.push_back(enhanced ? 1 : 0);
    }
    std::vector<int64_t> cptr((size_t)A.n + 1, 0);
    for (int64_t p = 0; p < nnz; ++p) cptr[A.colidx[p] + 1]++;
    for (int32_t j = 0; j < A.n; ++j) cptr[j + 1] += cptr[j];
    std::vector<int32_t> cp(nnz);
    std::vector<int64_t> fill(cptr.begin(), cptr.end() - 1);
    for (int64_t p = 0; p < nnz; ++p) cp[fill[A.colidx[p]]++] = (int32_t)p;
    for (int32_t j = 0; j < A.n; ++j) {
        if (cptr[j + 1] == cptr[j]) continue;
        s.H.pins.insert(s.H.pins.end(), cp.begin() + cptr[j], cp.begin() + cptr[j + 1]);
        s.H.xpins.push_back((int64_t)s.H.pins.size());
        s.H.nc.push_back(1);
        s.H.nrow.push_back(0);
    }
    s.H.nn = (int32_t)s.H.nc.size();
    s.H.build_vertex_side();
    return s;
}

// Split a subproblem along a bisection.  Cut nets are split (one net per
// side keeps the pins of that side); in the enhanced model cut row nets are
// removed with all their vertices.
void split_sub(Sub &S, const std::vector<uint8_t> &side, bool remove_cut_rows, Sub out[2],
               std::vector<int32_t> &removed) {
    const Hypergraph &H = S.H;
    std::vector<uint8_t> gone(H.nv, 0);
    if (remove_cut_rows) {
        for (int32_t n = 0; n < H.nn; ++n) {
            if (!H.nrow[n]) continue;
            bool s0 = false, s1 = false;
            for (int64_t p = H.xpins[n]; p < H.xpins[n + 1]; ++p) (side[H.pins[p]] ? s1 : s0) = true;
            if (s0 && s1)
                for (int64_t p = H.xpins[n]; p < H.xpins[n + 1]; ++p) gone[H.pins[p]] = 1;
        }
    }
    std::vector<int32_t> nid(H.nv, -1);
    for (int s = 0; s < 2; ++s) {
        out[s].H = Hypergraph();
        out[s].gid.clear();
    }
    for (int32_t v = 0; v < H.nv; ++v) {
        if (gone[v]) { removed.push_back(S.gid[v]); continue; }
        Sub &o = out[side[v]];
        nid[v] = (int32_t)o.gid.size();
        o.gid.push_back(S.gid[v]);
        o.H.vw.push_back(H.vw[v]);
    }
    for (int s = 0; s < 2; ++s) {
        out[s].H.nv = (int32_t)out[s].gid.size();
        out[s].H.xpins.push_back(0);
    }
    for (int32_t n = 0; n < H.nn; ++n) {
        for (int s = 0; s < 2; ++s) {
            Hypergraph &O = out[s].H;
            size_t before = O.pins.size();
            for (int64_t p = H.xpins[n]; p < H.xpins[n + 1]; ++p) {
                int32_t u = H.pins[p];
                if (!gone[u] && side[u] == s) O.pins.push_back(nid[u]);
            }
            if (O.pins.size() == before) continue;
            O.xpins.push_back((int64_t)O.pins.size());
            O.nc.push_back(H.nc[n]);
            O.nrow.push_back(H.nrow.empty() ? 0 : H.nrow[n]);
        }
    }
    for (int s = 0; s < 2; ++s) {
        out[s].H.nn = (int32_t)out[s].H.nc.size();
        out[s].H.build_vertex_side();
    }
    S.H = Hypergraph();
    S.gid.clear();
}

// Number of distinct vector entries a leaf touches: columns (SB/DB rows
// subproblem) or rows plus columns (split).  Every net of a subproblem has at
// least one pin, so this is the net count.
int64_t window_of(const Sub &S) { return S.H.nn; }

void recurse(Ctx &C, Sub S, int32_t K, int32_t part, uint64_t path, int32_t depth, bool leafmode);

void spawn_or_run(Ctx &C, Sub &&S, int32_t K, int32_t part, uint64_t path, int32_t depth,
                  bool leafmode, std::vector<std::future<void>> &futs) {
    bool big = S.H.nv > 20000;
    if (big && C.active.load() < num_threads()) {
        C.active++;
        futs.push_back(std::async(std::launch::async,
                                  [&C, K, part, path, depth, leafmode](Sub s) {
                                      recurse(C, std::move(s), K, part, path, depth, leafmode);
                                      C.active--;
                                  },
                                  std::move(S)));
    } else {
        recurse(C, std::move(S), K, part, path, depth, leafmode);
    }
}

void recurse(Ctx &C, Sub S, int32_t K, int32_t part, uint64_t path, int32_t depth, bool leafmode) {
    if (!leafmode && K == 1) {
        bool refine = C.window > 0;
        if (refine && C.model == Model::ERowColumnNet) {
            // leaves of a DB part: column-net model over the part's rows
            std::vector<int32_t> rows;
            rows.reserve(S.gid.size());
            std::vector<int32_t> nzs = S.gid;
            std::sort(nzs.begin(), nzs.end());
            // nonzero ids are in CSR order: map to rows
            const CsrHost &A = *C.A;
            int32_t r = 0;
            for (int32_t p : nzs) {
                while (A.rowptr[r + 1] <= p) ++r;
                if (rows.empty() || rows.back() != r) rows.push_back(r);
            }
            S = column_net_of_rows(A, rows);
        }
        if (refine) {
            recurse(C, std::move(S), 1, part, 0, 0, true);
        } else {
            std::lock_guard<std::mutex> g(C.mu);
            C.leaves.push_back(Leaf{part, 0, 0, std::move(S.gid)});
        }
        return;
    }
    if (leafmode) {
        bool stop = window_of(S) <= C.window || S.H.nv <= 1 || depth >= 20;
        if (stop) {
            std::lock_guard<std::mutex> g(C.mu);
            C.leaves.push_back(Leaf{part, path, depth, std::move(S.gid)});
            return;
        }
    }
    int32_t K0 = leafmode ? 1 : K / 2;
    int32_t K1 = leafmode ? 1 : K - K0;
    double frac0 = leafmode ? 0.5 : (double)K0 / (double)K;
    uint64_t sseed = mix(mix(C.seed, (uint64_t)part * 1315423911ull + (uint64_t)K),
                         path * 2654435761ull + (uint64_t)depth + (leafmode ? 77 : 0));
    std::vector<uint8_t> side;
    // this thread and the free slots
    const int32_t spare = std::max<int32_t>(1, num_threads() - C.active.load() + 1);
    int64_t c = bisect(S.H, frac0, C.eps, sseed, side, spare);
    if (!leafmode && C.model == Model::ERowColumnNet) {
        int64_t c0 = c;
        auto rows_cut = [&](int64_t &nnzc) {
            int64_t k = 0;
            nnzc = 0;
            for (int32_t n = 0; n < S.H.nn; ++n) {
                if (!S.H.nrow[n]) continue;
                bool a = false, b = false;
                for (int64_t p = S.H.xpins[n]; p < S.H.xpins[n + 1]; ++p) (side[S.H.pins[p]] ? b : a) = true;
                if (a && b) { ++k; nnzc += S.H.xpins[n + 1] - S.H.xpins[n]; }
            }
            return k;
        };
        int64_t z0 = 0, z1 = 0, k0 = 0, k1 = 0;
        bool dbg = getenv("SPX_DEBUG") && S.H.nv > 1000000;
        if (dbg) k0 = rows_cut(z0);
        c = uncut_rows(S.H, side, frac0, C.eps, c);
        if (dbg) {
            k1 = rows_cut(z1);
            fprintf(stderr, "  ercn nv=%d cut %lld -> %lld, cut rows %lld (%lld nnz) -> %lld (%lld nnz)\n", S.H.nv,
                    (long long)c0, (long long)c, (long long)k0, (long long)z0, (long long)k1, (long long)z1);
        }
    }
    if (!leafmode) C.cut += c;
    Sub out[2];
    std::vector<int32_t> removed;
    bool rem = (C.model == Model::ERowColumnNet) && !leafmode;
    split_sub(S, side, rem, out, removed);
    if (!removed.empty()) {
        std::lock_guard<std::mutex> g(C.mu);
        C.removed.insert(C.removed.end(), removed.begin(), removed.end());
    }
    if (leafmode && (out[0].gid.empty() || out[1].gid.empty())) {
        // the bisection could not separate anything: keep one leaf
        Sub &keep = out[0].gid.empty() ? out[1] : out[0];
        std::lock_guard<std::mutex> g(C.mu);
        C.leaves.push_back(Leaf{part, path, depth, std::move(keep.gid)});
        return;
    }
    // the first half goes to another thread when one is free, this thread
    // works on the second half and gives up its slot only while it waits
    std::vector<std::future<void>> futs;
    if (leafmode) {
        uint64_t bit = depth < 63 ? (1ull << (63 - depth)) : 0;
        spawn_or_run(C, std::move(out[0]), 1, part, path, depth + 1, true, futs);
        recurse(C, std::move(out[1]), 1, part, path | bit, depth + 1, true);
    } else {
        spawn_or_run(C, std::move(out[0]), K0, part, 0, depth + 1, false, futs);
        recurse(C, std::move(out[1]), K1, part + K0, 0, depth + 1, false);
    }
    if (!futs.empty()) {
        C.active--;
        for (auto &f : futs) f.get();
        C.active++;
    }
}

}  // namespace

// The row-net model of A is the column-net model of its transpose: the
// columns of A are partitioned; then each row lands in the one part its
// columns lie in, or in the row border (part K) when they lie in several
// (empty rows join part 0).  Leaves are the parts.
static PartitionResult partition_row_net(const CsrHost &A, int32_t K, uint64_t seed) {
    auto t0 = std::chrono::steady_clock::now();
    CsrHost At;
    At.m = A.n;
    At.n = A.m;
    At.nnz = A.nnz;
    At.rowptr.assign((size_t)A.n + 1, 0);
    for (int64_t q = 0; q < A.nnz; ++q) At.rowptr[A.colidx[q] + 1]++;
    for (int32_t j = 0; j < A.n; ++j) At.rowptr[j + 1] += At.rowptr[j];
    At.colidx.resize(A.nnz);
    {
        std::vector<int32_t> fill(At.rowptr.begin(), At.rowptr.end() - 1);
        for (int32_t i = 0; i < A.m; ++i)
            for (int32_t q = A.rowptr[i]; q < A.rowptr[i + 1]; ++q) At.colidx[fill[A.colidx[q]]++] = i;
    }
    PartitionResult c = partition(At, Model::ColumnNet, K, 0, seed);
    PartitionResult R;
    R.part.assign(A.m, 0);
    R.leaf.assign(A.m, 0);
    for (int32_t i = 0; i < A.m; ++i) {
        int32_t p = -1;
        bool cut = false;
        for (int32_t q = A.rowptr[i]; q < A.rowptr[i + 1]; ++q) {
            const int32_t pc = c.part[A.colidx[q]];
            if (p < 0) p = pc;
            else if (pc != p) cut = true;
        }
        R.part[i] = p < 0 ? 0 : (cut ? K : p);
        R.leaf[i] = R.part[i] < K ? R.part[i] : -1;
    }
    R.nleaves = K;
    R.cut = c.cut;
    R.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return R;
}

PartitionResult partition(const CsrHost &A, Model model, int32_t K, int64_t window_entries,
                          uint64_t seed, int64_t row_net_cost) {
    if (model == Model::RowNet) return partition_row_net(A, K, seed);
    auto t0 = std::chrono::steady_clock::now();
    Ctx C;
    C.model = model;
    C.K = K;
    C.window = window_entries;
    C.seed = seed;
    C.eps = 0.05;
    C.A = &A;
    Sub root;
    if (model == Model::ColumnNet) {
        std::vector<int32_t> rows(A.m);
        std::iota(rows.begin(), rows.end(), 0);
        root = column_net_of_rows(A, rows);
    } else {
        root = row_column_net(A, model == Model::ERowColumnNet, row_net_cost);
    }
    recurse(C, std::move(root), K, 0, 0, 0, false);

    PartitionResult R;
    // leaves numbered part-major, then by bisection path (side 0 first)
    std::sort(C.leaves.begin(), C.leaves.end(), [](const Leaf &a, const Leaf &b) {
        if (a.part != b.part) return a.part < b.part;
        return a.path < b.path;
    });
    bool rows_model = model != Model::RowColumnNet;
    size_t nitems = rows_model ? (size_t)A.m : (size_t)A.nnz;
    R.part.assign(nitems, -1);
    R.leaf.assign(nitems, -1);
    R.nleaves = (int32_t)C.leaves.size();
    if (model == Model::ERowColumnNet && C.window > 0) {
        // leaves hold rows already
        for (int32_t l = 0; l < R.nleaves; ++l)
            for (int32_t r : C.leaves[l].gid) {
                R.part[r] = C.leaves[l].part;
                R.leaf[r] = l;
            }
    } else if (model == Model::ERowColumnNet) {
        std::vector<int32_t> row_of(A.nnz);
        for (int32_t i = 0; i < A.m; ++i)
            for (int32_t p = A.rowptr[i]; p < A.rowptr[i + 1]; ++p) row_of[p] = i;
        for (int32_t l = 0; l < R.nleaves; ++l)
            for (int32_t p : C.leaves[l].gid) {
                R.part[row_of[p]] = C.leaves[l].part;
                R.leaf[row_of[p]] = l;
            }
    } else {
        for (int32_t l = 0; l < R.nleaves; ++l)
            for (int32_t g : C.leaves[l].gid) {
                R.part[g] = C.leaves[l].part;
                R.leaf[g] = l;
            }
    }
    if (model == Model::ERowColumnNet) {
        std::vector<int32_t> row_of_removed;
        for (int32_t p : C.removed) {
            int32_t i = (int32_t)(std::upper_bound(A.rowptr.begin(), A.rowptr.end(), p) -
                                  A.rowptr.begin()) - 1;
            R.part[i] = K;
            R.leaf[i] = -1;
        }
        // rows without nonzeros have no vertex: they join part 0's first leaf
        for (int32_t i = 0; i < A.m; ++i)
            if (R.part[i] < 0) {
                R.part[i] = 0;
                R.leaf[i] = 0;
            }
    }
    if (model == Model::ColumnNet) {
        for (int32_t i = 0; i < A.m; ++i)
            if (R.part[i] < 0) { R.part[i] = 0; R.leaf[i] = 0; }
    }
    R.cut = C.cut.load();
    R.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return R;
}

}  // namespace spx
