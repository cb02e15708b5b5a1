// Host-side mesh analysis: CSR structure of the node graph, greedy element
// colouring, and element validity checks.  Done once per mesh: the paper reuses
// the matrix structure across all time steps (Sec. III-B).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>

#include "internal.hpp"

namespace rafem {

namespace {

template <typename F>
void parallel_for(int64_t n, F&& f) {
    unsigned hw = std::thread::hardware_concurrency();
    int64_t nt = std::max<int64_t>(1, std::min<int64_t>(hw ? hw : 1, 16));
    if (n < 100000) nt = 1;
    if (nt == 1) {
        f(0, n);
        return;
    }
    std::vector<std::thread> th;
    int64_t chunk = (n + nt - 1) / nt;
    for (int64_t t = 0; t < nt; ++t) {
        int64_t lo = t * chunk, hi = std::min(n, lo + chunk);
        if (lo >= hi) break;
        th.emplace_back([&f, lo, hi] { f(lo, hi); });
    }
    for (auto& x : th) x.join();
}

// node -> incident elements, as CSR (n2e_ptr [n+1], n2e [E*npe])
void node_to_elements(int64_t n, int64_t E, int npe, const int32_t* conn,
                      std::vector<int64_t>& ptr, std::vector<int32_t>& adj) {
    ptr.assign(n + 1, 0);
    for (int64_t i = 0; i < E * npe; ++i) ptr[conn[i] + 1]++;
    for (int64_t i = 0; i < n; ++i) ptr[i + 1] += ptr[i];
    adj.resize(E * npe);
    std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
    for (int64_t e = 0; e < E; ++e)
        for (int a = 0; a < npe; ++a) adj[fill[conn[e * npe + a]]++] = (int32_t)e;
}

}  // namespace

void node_elements(int64_t n, int64_t E, int npe, const int32_t* conn, std::vector<int32_t>& ptr,
                   std::vector<int32_t>& list) {
    // CSR by node of the incidences (e, a) with conn[e][a] = node, packed as e npe + a, in
    // increasing element order
    std::vector<int64_t> p64;
    std::vector<int32_t> adj;
    node_to_elements(n, E, npe, conn, p64, adj);
    ptr.resize(n + 1);
    for (int64_t i = 0; i <= n; ++i) ptr[i] = (int32_t)p64[i];
    list.resize(adj.size());
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = p64[i]; k < p64[i + 1]; ++k) {
            const int32_t e = adj[k];
            int a = 0;
            while (conn[(int64_t)e * npe + a] != i) ++a;
            list[k] = e * npe + a;
        }
}

void check_conn(int64_t n_nodes, int64_t n_elems, int npe, const int32_t* conn) {
    if (n_nodes <= 0 || n_nodes > INT32_MAX - 1) throw Error{RAFEM_E_ARG, "n_nodes out of range"};
    if (n_elems <= 0 || n_elems > INT32_MAX / 8) throw Error{RAFEM_E_ARG, "n_elems out of range"};
    if (npe != 8 && npe != 4) throw Error{RAFEM_E_ARG, "nodes_per_elem must be 8 (hex) or 4 (tet)"};
    if (!conn) throw Error{RAFEM_E_ARG, "conn is NULL"};
    for (int64_t i = 0; i < n_elems * npe; ++i)
        if (conn[i] < 0 || conn[i] >= n_nodes)
            throw Error{RAFEM_E_MESH, "element " + std::to_string(i / npe) +
                                          " refers to node " + std::to_string(conn[i]) +
                                          " outside [0, n_nodes)"};
    for (int64_t e = 0; e < n_elems; ++e)
        for (int a = 0; a < npe; ++a)
            for (int b = a + 1; b < npe; ++b)
                if (conn[e * npe + a] == conn[e * npe + b])
                    throw Error{RAFEM_E_MESH, "element " + std::to_string(e) + " repeats a node"};
}

HostStructure build_structure(int64_t n, int64_t E, int npe, const int32_t* conn) {
    std::vector<int64_t> ptr;
    std::vector<int32_t> adj;
    node_to_elements(n, E, npe, conn, ptr, adj);

    // Pass 1: row lengths.  Pass 2: sorted unique columns.
    std::vector<int64_t> len(n + 1, 0);
    auto row_cols = [&](int64_t i, std::vector<int32_t>& buf) {
        buf.clear();
        for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) {
            const int32_t* el = conn + (int64_t)adj[k] * npe;
            for (int a = 0; a < npe; ++a) buf.push_back(el[a]);
        }
        std::sort(buf.begin(), buf.end());
        buf.erase(std::unique(buf.begin(), buf.end()), buf.end());
    };
    parallel_for(n, [&](int64_t lo, int64_t hi) {
        std::vector<int32_t> buf;
        for (int64_t i = lo; i < hi; ++i) {
            row_cols(i, buf);
            if (buf.empty()) buf.push_back((int32_t)i);  // isolated node: keep a diagonal
            len[i + 1] = (int64_t)buf.size();
        }
    });
    for (int64_t i = 0; i < n; ++i) len[i + 1] += len[i];
    if (len[n] > INT32_MAX) throw Error{RAFEM_E_MESH, "nnz exceeds INT32_MAX"};
    HostStructure S;
    S.row_ptr.resize(n + 1);
    for (int64_t i = 0; i <= n; ++i) S.row_ptr[i] = (int32_t)len[i];
    S.col_idx.resize(len[n]);
    parallel_for(n, [&](int64_t lo, int64_t hi) {
        std::vector<int32_t> buf;
        for (int64_t i = lo; i < hi; ++i) {
            row_cols(i, buf);
            if (buf.empty()) buf.push_back((int32_t)i);
            std::memcpy(S.col_idx.data() + len[i], buf.data(), buf.size() * sizeof(int32_t));
        }
    });
    return S;
}

HostSell build_sell(const HostStructure& S, int64_t n, const std::vector<int64_t>& row_off) {
    // Slabs of 64 consecutive rows, one row per lane of a wavefront.  Entry j of row r
    // lives at sptr[r / 64] + (r % 64) + 64 j, so a wavefront reading entry j of its 64
    // rows touches 64 consecutive words.  A slab is as wide as its longest row.
    //
    // Shared-offset slabs: when the column offsets (column - row) of a full slab's rows
    // together take no more distinct values than the slab is wide, entry j of every row
    // of the slab is given the same offset U[j] (U sorted ascending), its value being 0
    // where (r, r + U[j]) is not an entry of the matrix.  The SpMV then reads one offset
    // list per slab instead of one offset per entry, and its x reads are contiguous.  This
    // holds for every slab of the grid meshes away from the first and last planes (rows
    // on a boundary have a subset of the interior stencil).  Every r + U[j] must lie in
    // the rows of the slab's own sample (row_off), so a slab never reads another sample.
    //
    // Other slabs: shorter rows are padded with value 0 and their own row index as column
    // (a valid x index).  In both kinds the columns of a row ascend along its entries.
    HostSell L;
    L.nslabs = (n + 63) / 64;
    L.sptr.assign(L.nslabs + 1, 0);
    L.sofs.assign(L.nslabs, -1);
    L.rlen.assign(n, 0);
    std::vector<std::vector<int32_t>> shared(L.nslabs);
    std::vector<int32_t> width(L.nslabs, 0);
    parallel_for(L.nslabs, [&](int64_t s_lo, int64_t s_hi) {
        std::vector<int32_t> U;
        for (int64_t s = s_lo; s < s_hi; ++s) {
            const int64_t r0 = s * 64, r1 = std::min<int64_t>(n, r0 + 64);
            int32_t w = 0;
            for (int64_t r = r0; r < r1; ++r) w = std::max(w, S.row_ptr[r + 1] - S.row_ptr[r]);
            width[s] = w;
            // the sample holding row r0
            const size_t q = (size_t)(std::upper_bound(row_off.begin(), row_off.end(), r0) -
                                      row_off.begin()) - 1;
            const int64_t lo = row_off[q], hi = row_off[q + 1];
            if (r1 - r0 != 64 || r1 > hi) continue;
            U.clear();
            for (int64_t r = r0; r < r1; ++r)
                for (int32_t k = S.row_ptr[r]; k < S.row_ptr[r + 1]; ++k)
                    U.push_back((int32_t)(S.col_idx[k] - r));
            std::sort(U.begin(), U.end());
            U.erase(std::unique(U.begin(), U.end()), U.end());
            bool ok = (int32_t)U.size() <= w;
            for (size_t j = 0; ok && j < U.size(); ++j)
                ok = r0 + U[j] >= lo && r1 - 1 + U[j] < hi;
            if (ok) {
                width[s] = (int32_t)U.size();
                shared[s] = U;
            }
        }
    });
    int64_t total = 0;
    for (int64_t s = 0; s < L.nslabs; ++s) {
        total += 64 * (int64_t)width[s];
        if (total > INT32_MAX) throw Error{RAFEM_E_MESH, "padded slab storage exceeds INT32_MAX"};
        L.sptr[s + 1] = (int32_t)total;
        if (!shared[s].empty()) {
            L.sofs[s] = (int32_t)L.soff.size();
            L.soff.insert(L.soff.end(), shared[s].begin(), shared[s].end());
        }
    }
    L.scol.assign(total, 0);
    parallel_for(L.nslabs, [&](int64_t s_lo, int64_t s_hi) {
        for (int64_t s = s_lo; s < s_hi; ++s) {
            const int32_t base = L.sptr[s];
            const int32_t w = (L.sptr[s + 1] - base) / 64;
            if (!shared[s].empty()) {
                const std::vector<int32_t>& U = shared[s];
                for (int64_t lane = 0; lane < 64; ++lane) {
                    const int64_t r = s * 64 + lane;
                    L.rlen[r] = w;
                    for (int32_t j = 0; j < w; ++j)
                        L.scol[base + lane + 64 * (int64_t)j] = (int32_t)(r + U[j]);
                }
                continue;
            }
            for (int64_t lane = 0; lane < 64; ++lane) {
                const int64_t r = s * 64 + lane;
                const int32_t pad = (int32_t)std::min<int64_t>(r, n - 1);
                int32_t len = 0;
                if (r < n) {
                    len = S.row_ptr[r + 1] - S.row_ptr[r];
                    L.rlen[r] = len;
                    for (int32_t j = 0; j < len; ++j)
                        L.scol[base + lane + 64 * (int64_t)j] = S.col_idx[S.row_ptr[r] + j];
                }
                for (int32_t j = len; j < w; ++j) L.scol[base + lane + 64 * (int64_t)j] = pad;
            }
        }
    });
    // 16-bit offsets to the row (padding: offset 0) for every slab without a shared list
    // whose columns are all within reach of its rows; the others keep their 32-bit columns
    // (sofs = -2).  No such slab within reach: no offsets at all.
    std::vector<uint8_t> near(L.nslabs, 0);
    parallel_for(L.nslabs, [&](int64_t s_lo, int64_t s_hi) {
        for (int64_t s = s_lo; s < s_hi; ++s) {
            if (L.sofs[s] >= 0) continue;
            bool ok = true;
            for (int64_t k = L.sptr[s]; ok && k < L.sptr[s + 1]; ++k) {
                const int64_t r = std::min<int64_t>(s * 64 + (k - L.sptr[s]) % 64, n - 1);
                const int64_t d = (int64_t)L.scol[k] - r;
                ok = d >= INT16_MIN && d <= INT16_MAX;
            }
            near[s] = ok ? 1 : 0;
        }
    });
    if (std::find(near.begin(), near.end(), 1) != near.end()) {
        L.sdel.assign(total, 0);
        parallel_for(L.nslabs, [&](int64_t s_lo, int64_t s_hi) {
            for (int64_t s = s_lo; s < s_hi; ++s) {
                if (L.sofs[s] >= 0) continue;
                if (!near[s]) {
                    L.sofs[s] = -2;
                    continue;
                }
                for (int64_t k = L.sptr[s]; k < L.sptr[s + 1]; ++k) {
                    const int64_t r = std::min<int64_t>(s * 64 + (k - L.sptr[s]) % 64, n - 1);
                    L.sdel[k] = (int16_t)((int64_t)L.scol[k] - r);
                }
            }
        });
    }
    return L;
}

int colour_elements(int64_t n, int64_t E, int npe, const int32_t* conn, int32_t* colour) {
    // Greedy first fit in element order.  mask[node] holds the colours of the already
    // coloured elements that touch the node (kColourWords x 64 bits); an element takes the
    // lowest colour absent from the union of its nodes' masks, so no two elements of one
    // colour share a node.
    std::vector<uint64_t> mask((size_t)n * kColourWords, 0);
    int used = 0;
    for (int64_t e = 0; e < E; ++e) {
        const int32_t* el = conn + e * npe;
        uint64_t taken[kColourWords] = {};
        for (int a = 0; a < npe; ++a)
            for (int w = 0; w < kColourWords; ++w) taken[w] |= mask[(size_t)el[a] * kColourWords + w];
        int c = -1;
        for (int w = 0; w < kColourWords && c < 0; ++w)
            if (taken[w] != ~0ull) c = 64 * w + __builtin_ctzll(~taken[w]);
        if (c < 0)
            throw Error{RAFEM_E_MESH, "element colouring needs more than " +
                                          std::to_string(64 * kColourWords) + " colours"};
        colour[e] = c;
        used = std::max(used, c + 1);
        for (int a = 0; a < npe; ++a) mask[(size_t)el[a] * kColourWords + c / 64] |= 1ull << (c % 64);
    }
    return used;
}

void degree_sort(int64_t n, const HostStructure& S, int64_t window, int32_t* order) {
    // Within consecutive windows of positions, nodes by increasing degree (row length less
    // the diagonal), ties in their current order: each slab of 64 rows then holds rows of
    // nearly equal length, so little of it is padding.
    std::vector<int32_t> seg;
    for (int64_t s0 = 0; s0 < n; s0 += window) {
        const int64_t s1 = std::min(n, s0 + window);
        seg.assign(order + s0, order + s1);
        std::stable_sort(seg.begin(), seg.end(), [&](int32_t a, int32_t b) {
            return S.row_ptr[a + 1] - S.row_ptr[a] < S.row_ptr[b + 1] - S.row_ptr[b];
        });
        std::copy(seg.begin(), seg.end(), order + s0);
    }
}

std::vector<int32_t> rcm_order(int64_t n, const HostStructure& S) {
    // Reverse Cuthill-McKee on the node graph (neighbours: the row's columns without the
    // diagonal).  Per component, in order of its smallest node id: the pseudo-peripheral
    // start node of George and Liu (from the node of least degree, move to the least-degree
    // node of the last BFS level while the number of levels grows; ties: smallest id), then
    // breadth-first search taking unvisited neighbours by increasing degree (ties: smallest
    // id); finally the whole order is reversed.
    auto deg = [&](int64_t v) { return S.row_ptr[v + 1] - S.row_ptr[v] - 1; };
    auto less = [&](int32_t a, int32_t b) { return deg(a) != deg(b) ? deg(a) < deg(b) : a < b; };
    std::vector<int32_t> order;
    order.reserve(n);
    std::vector<char> visited(n, 0);
    std::vector<int32_t> mark(n, 0);  // BFS stamps
    int32_t stamp = 0;
    std::vector<int32_t> comp, cur, nxt;
    // levels of a BFS from r: returns their number; cur holds the last level
    auto levels = [&](int32_t r) {
        ++stamp;
        mark[r] = stamp;
        cur.assign(1, r);
        int nlev = 1;
        for (;;) {
            nxt.clear();
            for (int32_t v : cur)
                for (int32_t k = S.row_ptr[v]; k < S.row_ptr[v + 1]; ++k) {
                    const int32_t w = S.col_idx[k];
                    if (mark[w] != stamp) {
                        mark[w] = stamp;
                        nxt.push_back(w);
                    }
                }
            if (nxt.empty()) return nlev;
            cur.swap(nxt);
            ++nlev;
        }
    };
    for (int64_t seed = 0; seed < n; ++seed) {
        if (visited[seed]) continue;
        // the component of seed
        ++stamp;
        mark[seed] = stamp;
        comp.assign(1, (int32_t)seed);
        for (size_t i = 0; i < comp.size(); ++i) {
            const int32_t v = comp[i];
            for (int32_t k = S.row_ptr[v]; k < S.row_ptr[v + 1]; ++k) {
                const int32_t w = S.col_idx[k];
                if (mark[w] != stamp) {
                    mark[w] = stamp;
                    comp.push_back(w);
                }
            }
        }
        int32_t r = *std::min_element(comp.begin(), comp.end(), less);
        int nlev = levels(r);
        for (;;) {
            const int32_t cand = *std::min_element(cur.begin(), cur.end(), less);
            const int nl = levels(cand);
            if (nl > nlev) {
                r = cand;
                nlev = nl;
            } else {
                break;
            }
        }
        // Cuthill-McKee from r
        size_t head = order.size();
        visited[r] = 1;
        order.push_back(r);
        std::vector<int32_t> fresh;
        while (head < order.size()) {
            const int32_t v = order[head++];
            fresh.clear();
            for (int32_t k = S.row_ptr[v]; k < S.row_ptr[v + 1]; ++k) {
                const int32_t w = S.col_idx[k];
                if (!visited[w]) {
                    visited[w] = 1;
                    fresh.push_back(w);
                }
            }
            std::sort(fresh.begin(), fresh.end(), less);
            order.insert(order.end(), fresh.begin(), fresh.end());
        }
    }
    std::reverse(order.begin(), order.end());
    return order;
}

bool check_geometry(int64_t E, int npe, const int32_t* conn, const double* xyz) {
    // Reference-cube corner signs of the 8 hex nodes (local order of the ABI).
    static const double sx[8] = {-1, 1, 1, -1, -1, 1, 1, -1};
    static const double sy[8] = {-1, -1, 1, 1, -1, -1, 1, 1};
    static const double sz[8] = {-1, -1, -1, -1, 1, 1, 1, 1};
    const double g = 1.0 / std::sqrt(3.0);
    std::atomic<int64_t> bad{-1};
    std::atomic<bool> affine{true};
    parallel_for(E, [&](int64_t lo, int64_t hi) {
        bool aff = true;
        for (int64_t e = lo; e < hi; ++e) {
            const int32_t* el = conn + e * npe;
            bool ok = true;
            if (npe == 8 && aff) {
                // parallelepiped: every corner is x0 + o1 (x1-x0) + o2 (x3-x0) + o3 (x4-x0)
                double scale = 0.0;
                for (int i = 0; i < 3; ++i) {
                    scale = std::max(scale, std::fabs(xyz[el[1] * 3 + i] - xyz[el[0] * 3 + i]));
                    scale = std::max(scale, std::fabs(xyz[el[3] * 3 + i] - xyz[el[0] * 3 + i]));
                    scale = std::max(scale, std::fabs(xyz[el[4] * 3 + i] - xyz[el[0] * 3 + i]));
                }
                for (int a = 0; a < 8 && aff; ++a) {
                    const double o1 = sx[a] > 0, o2 = sy[a] > 0, o3 = sz[a] > 0;
                    for (int i = 0; i < 3; ++i) {
                        const double x0 = xyz[el[0] * 3 + i];
                        const double pred = x0 + o1 * (xyz[el[1] * 3 + i] - x0) +
                                            o2 * (xyz[el[3] * 3 + i] - x0) +
                                            o3 * (xyz[el[4] * 3 + i] - x0);
                        if (std::fabs(xyz[el[a] * 3 + i] - pred) > 1e-12 * scale) aff = false;
                    }
                }
            }
            if (npe == 4) {
                double J[3][3];
                for (int c = 0; c < 3; ++c)
                    for (int i = 0; i < 3; ++i) J[i][c] = xyz[el[c + 1] * 3 + i] - xyz[el[0] * 3 + i];
                double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                             J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                             J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
                ok = det > 0;
            } else {
                for (int q = 0; q < 8 && ok; ++q) {
                    double xi = sx[q] * g, et = sy[q] * g, ze = sz[q] * g;
                    double J[3][3] = {{0}};
                    for (int a = 0; a < 8; ++a) {
                        double d0 = 0.125 * sx[a] * (1 + sy[a] * et) * (1 + sz[a] * ze);
                        double d1 = 0.125 * sy[a] * (1 + sx[a] * xi) * (1 + sz[a] * ze);
                        double d2 = 0.125 * sz[a] * (1 + sx[a] * xi) * (1 + sy[a] * et);
                        for (int i = 0; i < 3; ++i) {
                            double x = xyz[el[a] * 3 + i];
                            J[i][0] += x * d0;
                            J[i][1] += x * d1;
                            J[i][2] += x * d2;
                        }
                    }
                    double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                                 J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                                 J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
                    ok = det > 0;
                }
            }
            if (!ok) {
                bad.store(e);  // any offending element will do for the message
                return;
            }
        }
        if (!aff) affine.store(false);
    });
    if (bad.load() >= 0)
        throw Error{RAFEM_E_MESH, "element " + std::to_string(bad.load()) +
                                      " has a non-positive Jacobian determinant"};
    return affine.load();
}

}  // namespace rafem
