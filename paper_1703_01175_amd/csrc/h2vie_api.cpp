// Host side of the C ABI declared in include/h2vie.h: validation of the host
// description, packing into the caller's device buffer, handles, dispatch.
#include <hip/hip_runtime.h>

#include <atomic>
#include <thread>

#include <algorithm>
#include <cstdarg>
#include <map>
#include <mutex>
#include <set>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/h2vie.h"
#include "h2_internal.h"
#include "h2_api_internal.h"

using namespace h2;

namespace {

thread_local std::string g_last_error;

h2_status fail(h2_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
h2_status fail(h2_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}


// Planned layout: every array at a 256-byte aligned offset of the device buffer.
struct Layout {
    size_t total = 0;
    size_t add(size_t bytes) {
        size_t off = total;
        total += (bytes + 255) & ~size_t(255);
        return off;
    }
};

struct Plan {
    // host staging (int arrays) and device offsets
    std::vector<int> perm, cl_rank, cl_coef, cl_begin, cl_size, cl_parent, cl_first_child, cl_nchild;
    std::vector<int64_t> cl_toff, cl_boff;
    std::vector<int> leaf_id, near_ptr, near_sbeg, near_ssize;
    std::vector<int64_t> near_off;
    // near blocks as held on the device: offset of each near pair's block in the stored
    // array, and the source block of every stored one (identical blocks stored once)
    std::vector<int64_t> near_uoff;
    std::vector<int64_t> near_src;
    int64_t near_stored_len = 0;
    bool near_dedup = false;
    // stored-once near blocks split into passes of about kNearPassBytes of distinct blocks
    // each (so one pass's blocks stay in an XCD's L2); pass p of launch slot q covers the
    // list entries [near_pass_ptr[q (P + 1) + p], near_pass_ptr[q (P + 1) + p + 1])
    int near_passes = 1;
    std::vector<int> near_pass_ptr;
    size_t o_npass = 0, o_ypart = 0;
    // tiled near field over stored-once blocks (see DevH2): tiles of kTileLeaves leaves
    // consecutive in tree order, each with its steps (one stored block, per target slot a
    // source); every tile walks the stored blocks in the same order
    std::vector<int> tile_ptr, tile_leaf, step_shape, step_src;
    std::vector<int64_t> step_off;
    int64_t tile_pairs = 0;
    size_t o_tile[4] = {0, 0, 0, 0}, o_stepoff = 0, o_tzero = 0, o_tpart1 = 0;
    // symmetric near field: each unordered leaf pair once (empty when G_st != G_ts^T somewhere)
    bool sym = false;
    int64_t sym_pairs = 0;
    std::vector<int> sym_leaf, sym_ptr, sym_sbeg, sym_ssize, sym_pslot, sym_in_ptr, sym_in_slot;
    std::vector<int64_t> sym_off;
    size_t o_sym[7] = {0, 0, 0, 0, 0, 0, 0}, o_symoff = 0, o_sympart = 0, o_symrows = 0;
    std::vector<int> row_cl, row_ncols, row_colptr, colsrc;
    std::vector<int64_t> row_off;

    // symmetric couplings (empty when S_st != S_ts^T somewhere): each unordered admissible
    // pair streamed once by its owner; per row slot the owned columns (their storage
    // column in the grouped row and coefficient row), their first partial column, and the
    // partial columns (first column of each block) that land in the slot's cluster
    bool csym = false;
    std::vector<int> row_nown, row_pbase, crecv_ptr, crecv_p;
    std::vector<int64_t> coup_dev_off;      // per far pair: element offset of its block on the device
    int64_t csym_elems = 0, csym_cols = 0;
    size_t o_csym[4] = {0, 0, 0, 0}, o_cpart = 0;
    std::vector<int> up_list, down_list;
    std::vector<int> lc_beg, lc_size;           // leaves in cluster order
    std::vector<int64_t> lc_diag, lc_inv;
    int64_t lc_inv_elems = 0;
    int lc_max = 0;
    size_t o_lbeg = 0, o_lsize = 0, o_ldiag = 0, o_linv = 0;
    LevelLaunch lv;
    int coef_rows = 0, depth = 0, max_rank = 0, min_leaf_rank = 1 << 30;
    int tiers = 1;
    // device offsets
    size_t o_perm, o_chi, o_cl[7], o_toff, o_boff, o_leaf, o_nptr, o_nsb, o_nss, o_noff;
    size_t o_rowcl, o_rownc, o_rowcp, o_colsrc, o_rowoff, o_up, o_down;
    size_t o_data[3][4];      // tier x {near, coupling, basis, transfer}
    // batched BF16x3 tier
    BatchHost* batch = nullptr;
    size_t o_arena = 0, o_ub = 0, o_xb = 0, o_yhb = 0, o_xf = 0, o_yhf = 0, o_yf = 0, o_prow = 0, o_jobs = 0, o_group = 0;
    size_t group_bytes = 0;
    ~Plan() { delete batch; }
    size_t o_U, o_X, o_Y, o_aux;
    int vec_cols = kNcomp;
    size_t aux_bytes = 0;
    Layout lay;
};

inline bool bad_ptr(const void* p) { return p == nullptr; }

h2_status validate(const h2_host_desc* d) {
    if (!d) return fail(H2_ERR_INVALID_ARG, "null host description");
    if (d->ncomp != kNcomp) return fail(H2_ERR_BAD_DESC, "ncomp must be 3 (got %d)", d->ncomp);
    if (d->n_vox <= 0 || d->n_vox >= (int64_t(1) << 31)) return fail(H2_ERR_BAD_DESC, "n_vox out of range");
    if (d->n_clusters <= 0) return fail(H2_ERR_BAD_DESC, "n_clusters must be positive");
    if (bad_ptr(d->perm) || bad_ptr(d->level) || bad_ptr(d->parent) || bad_ptr(d->begin) || bad_ptr(d->end) ||
        bad_ptr(d->first_child) || bad_ptr(d->nchild) || bad_ptr(d->rank) || bad_ptr(d->basis_off) ||
        bad_ptr(d->transfer_off) || bad_ptr(d->chi))
        return fail(H2_ERR_INVALID_ARG, "null array in host description");
    if ((d->n_far > 0 && (bad_ptr(d->far_t) || bad_ptr(d->far_s) || bad_ptr(d->far_off) || bad_ptr(d->coupling))) ||
        (d->n_near > 0 && (bad_ptr(d->near_t) || bad_ptr(d->near_s) || bad_ptr(d->near_off) || bad_ptr(d->near_blocks))) ||
        (d->basis_len > 0 && bad_ptr(d->basis)) || (d->transfer_len > 0 && bad_ptr(d->transfer)))
        return fail(H2_ERR_INVALID_ARG, "null block array in host description");
    if (d->n_far < 0 || d->n_near <= 0 || d->basis_len < 0 || d->transfer_len < 0 || d->coupling_len < 0 ||
        d->near_len <= 0)
        return fail(H2_ERR_BAD_DESC, "negative or empty sizes");
    if (!std::isfinite(d->k) || !std::isfinite(d->volume) || !std::isfinite(d->sigma) || d->volume <= 0)
        return fail(H2_ERR_BAD_DESC, "k, volume, sigma must be finite (volume > 0)");
    const int64_t n = d->n_vox;
    const int nc = d->n_clusters;
    {
        std::vector<char> seen(n, 0);
        for (int64_t p = 0; p < n; ++p) {
            int64_t v = d->perm[p];
            if (v < 0 || v >= n || seen[v]) return fail(H2_ERR_BAD_DESC, "perm is not a permutation (position %lld)", (long long)p);
            seen[v] = 1;
        }
    }
    if (d->parent[0] != -1 || d->begin[0] != 0 || d->end[0] != n || d->level[0] != 0)
        return fail(H2_ERR_BAD_DESC, "cluster 0 must be the root covering [0, n_vox)");
    for (int c = 0; c < nc; ++c) {
        if (d->begin[c] < 0 || d->end[c] > n || d->begin[c] >= d->end[c])
            return fail(H2_ERR_BAD_DESC, "cluster %d has an invalid range", c);
        if (d->rank[c] < 0 || d->rank[c] > kMaxRank) return fail(H2_ERR_BAD_DESC, "cluster %d rank out of [0, 256]", c);
        if (c > 0) {
            int p = d->parent[c];
            if (p < 0 || p >= c) return fail(H2_ERR_BAD_DESC, "cluster %d parent must precede it", c);
            if (d->level[c] != d->level[p] + 1) return fail(H2_ERR_BAD_DESC, "cluster %d level inconsistent", c);
        }
        if (d->level[c] < 0 || d->level[c] >= 63) return fail(H2_ERR_BAD_DESC, "cluster %d level out of range", c);
        if (d->nchild[c] == 0) {
            if (d->end[c] - d->begin[c] > kMaxLeaf) return fail(H2_ERR_BAD_DESC, "leaf %d larger than 64 voxels", c);
            if (d->rank[c] > 0) {
                int64_t o = d->basis_off[c];
                int64_t need = (d->end[c] - d->begin[c]) * d->rank[c];
                if (d->rank[c] > d->end[c] - d->begin[c]) return fail(H2_ERR_BAD_DESC, "leaf %d rank exceeds its size", c);
                if (o < 0 || o + need > d->basis_len) return fail(H2_ERR_BAD_DESC, "leaf %d basis offset out of range", c);
            }
        } else {
            int f = d->first_child[c], k = d->nchild[c];
            if (k < 0 || f <= c || f + k > nc) return fail(H2_ERR_BAD_DESC, "cluster %d children out of range", c);
            int64_t pos = d->begin[c];
            for (int ch = f; ch < f + k; ++ch) {
                if (d->parent[ch] != c || d->begin[ch] != pos)
                    return fail(H2_ERR_BAD_DESC, "children of %d do not tile its range", c);
                pos = d->end[ch];
            }
            if (pos != d->end[c]) return fail(H2_ERR_BAD_DESC, "children of %d do not tile its range", c);
        }
        if (c > 0) {
            int p = d->parent[c];
            if (d->rank[c] > 0 && d->rank[p] > 0) {
                int64_t o = d->transfer_off[c];
                int64_t need = int64_t(d->rank[c]) * d->rank[p];
                if (o < 0 || o + need > d->transfer_len) return fail(H2_ERR_BAD_DESC, "transfer of %d out of range", c);
            }
        }
    }
    // far pairs: grouped by row cluster, contiguous grouped block rows
    {
        std::vector<char> done(nc, 0);
        int64_t i = 0;
        while (i < d->n_far) {
            int t = d->far_t[i];
            if (t < 0 || t >= nc) return fail(H2_ERR_BAD_DESC, "far pair %lld: row cluster out of range", (long long)i);
            if (done[t]) return fail(H2_ERR_BAD_DESC, "far pairs of cluster %d are not consecutive", t);
            done[t] = 1;
            int kt = d->rank[t];
            if (kt <= 0) return fail(H2_ERR_BAD_DESC, "far pair %lld: row cluster %d has rank 0", (long long)i, t);
            int64_t off = d->far_off[i];
            for (; i < d->n_far && d->far_t[i] == t; ++i) {
                int s = d->far_s[i];
                if (s < 0 || s >= nc) return fail(H2_ERR_BAD_DESC, "far pair %lld: column cluster out of range", (long long)i);
                if (d->rank[s] <= 0) return fail(H2_ERR_BAD_DESC, "far pair %lld: column cluster %d has rank 0", (long long)i, s);
                if (d->far_off[i] != off)
                    return fail(H2_ERR_BAD_DESC, "far pair %lld: coupling blocks of row %d are not back to back", (long long)i, t);
                off += int64_t(kt) * d->rank[s];
                if (d->far_off[i] < 0 || off > d->coupling_len)
                    return fail(H2_ERR_BAD_DESC, "far pair %lld: coupling offset out of range", (long long)i);
            }
        }
    }
    for (int64_t i = 0; i < d->n_near; ++i) {
        int t = d->near_t[i], s = d->near_s[i];
        if (t < 0 || t >= nc || s < 0 || s >= nc) return fail(H2_ERR_BAD_DESC, "near pair %lld out of range", (long long)i);
        if (d->nchild[t] != 0 || d->nchild[s] != 0) return fail(H2_ERR_BAD_DESC, "near pair %lld is not leaf-leaf", (long long)i);
        if (i > 0 && d->near_t[i - 1] > t) return fail(H2_ERR_BAD_DESC, "near pairs are not sorted by row cluster");
        int64_t need = (d->end[t] - d->begin[t]) * (d->end[s] - d->begin[s]);
        if (d->near_off[i] < 0 || d->near_off[i] + need > d->near_len)
            return fail(H2_ERR_BAD_DESC, "near pair %lld: block offset out of range", (long long)i);
    }
    return H2_OK;
}

// Identical near blocks stored once.  A 64-bit hash of every block (host threads)
// proposes the matches, each confirmed bit for bit against the block it would
// share storage with; a block whose hash matches but whose entries differ keeps
// its own copy.  Kept only when the stored entries are at most half of them all.
static void plan_near_dedup(const h2_host_desc* d, bool allow, Plan& P) {
    const int64_t nn = d->n_near;
    auto bsize = [&](int64_t i) {
        return (d->end[d->near_t[i]] - d->begin[d->near_t[i]]) * (d->end[d->near_s[i]] - d->begin[d->near_s[i]]);
    };
    auto identity = [&]() {
        P.near_uoff.assign(d->near_off, d->near_off + nn);
        P.near_src.clear();
        P.near_stored_len = d->near_len;
        P.near_dedup = false;
    };
    if (!allow || nn == 0) {
        identity();
        return;
    }
    std::vector<uint64_t> hash(nn);
    auto hash_range = [&](int64_t a, int64_t b) {
        for (int64_t i = a; i < b; ++i) {
            const uint64_t* w = reinterpret_cast<const uint64_t*>(d->near_blocks + 2 * d->near_off[i]);
            const int64_t nw = 2 * bsize(i);
            uint64_t h = 0x9e3779b97f4a7c15ull ^ uint64_t(nw);
            for (int64_t k = 0; k < nw; ++k) {
                h ^= w[k];
                h *= 0x100000001b3ull;
                h ^= h >> 29;
            }
            hash[i] = h;
        }
    };
    const int64_t nth = std::max<int64_t>(1, std::min<int64_t>(8, nn / 1024 + 1));
    {
        std::vector<std::thread> th;
        for (int64_t k = 0; k < nth; ++k) th.emplace_back(hash_range, nn * k / nth, nn * (k + 1) / nth);
        for (auto& x : th) x.join();
    }
    // representative of each (size, hash): the first block that has it
    std::map<std::pair<int64_t, uint64_t>, int64_t> first;
    std::vector<int64_t> rep(nn);
    for (int64_t i = 0; i < nn; ++i) {
        auto it = first.emplace(std::make_pair(bsize(i), hash[i]), i).first;
        rep[i] = it->second;
    }
    // confirm every match bit for bit
    std::vector<char> same(nn, 1);
    auto confirm = [&](int64_t a, int64_t b) {
        for (int64_t i = a; i < b; ++i)
            if (rep[i] != i)
                same[i] = std::memcmp(d->near_blocks + 2 * d->near_off[i], d->near_blocks + 2 * d->near_off[rep[i]],
                                      size_t(bsize(i)) * 16) == 0;
    };
    {
        std::vector<std::thread> th;
        for (int64_t k = 0; k < nth; ++k) th.emplace_back(confirm, nn * k / nth, nn * (k + 1) / nth);
        for (auto& x : th) x.join();
    }
    P.near_uoff.assign(nn, -1);
    P.near_src.clear();
    int64_t stored = 0;
    for (int64_t i = 0; i < nn; ++i) {
        if (rep[i] != i && same[i]) {
            P.near_uoff[i] = P.near_uoff[rep[i]];
            continue;
        }
        P.near_uoff[i] = stored;
        P.near_src.push_back(i);
        stored += bsize(i);
    }
    if (2 * stored > d->near_len) {
        identity();
        return;
    }
    P.near_stored_len = stored;
    P.near_dedup = true;
}

// Symmetric near field.  G is symmetric (G_ij = G_ji), so when the description's
// blocks satisfy G_st = G_ts^T bit for bit, each unordered leaf pair {t, s} is
// streamed once by one of its two leaves (the owner, chosen to balance the blocks
// per leaf): the owner adds G_ts u_s to its own rows and writes G_ts^T u_t for
// the other leaf into a partial slot, which that leaf adds when it finishes.
// Diagonal blocks stay with their leaf.  Any asymmetric or unmatched pair leaves
// the plan without this mode.
static void plan_symmetric_near(const h2_host_desc* d, const std::vector<int64_t>& nfirst,
                                const std::vector<int64_t>& ncount, Plan& P) {
    const int nc = d->n_clusters;
    auto size = [&](int c) { return int(d->end[c] - d->begin[c]); };
    // mirror of every off-diagonal pair (t, s), t < s
    struct Pair { int t, s; int64_t it, is; };     // near index of (t, s) and of (s, t)
    std::vector<Pair> pairs;
    for (int t = 0; t < nc; ++t) {
        if (d->nchild[t] != 0) continue;
        for (int64_t i = nfirst[t]; i < nfirst[t] + ncount[t]; ++i) {
            const int s = d->near_s[i];
            if (s <= t) continue;
            int64_t j = -1;
            for (int64_t k = nfirst[s]; k < nfirst[s] + ncount[s]; ++k)
                if (d->near_s[k] == t) { j = k; break; }
            if (j < 0) return;
            pairs.push_back({t, s, i, j});
        }
    }
    // bitwise check G_st = G_ts^T, pairs split over host threads
    std::atomic<bool> same(true);
    auto check = [&](size_t a, size_t b) {
        for (size_t q = a; q < b && same.load(std::memory_order_relaxed); ++q) {
            const Pair& pr = pairs[q];
            const int nt = size(pr.t), ns = size(pr.s);
            const double* gts = d->near_blocks + 2 * d->near_off[pr.it];   // nt x ns, column major
            const double* gst = d->near_blocks + 2 * d->near_off[pr.is];   // ns x nt, column major
            for (int b2 = 0; b2 < ns; ++b2)
                for (int a2 = 0; a2 < nt; ++a2)
                    if (std::memcmp(gts + 2 * (int64_t(b2) * nt + a2), gst + 2 * (int64_t(a2) * ns + b2), 16) != 0) {
                        same.store(false);
                        return;
                    }
        }
    };
    const size_t nth = std::max<size_t>(1, std::min<size_t>(8, pairs.size() / 4096 + 1));
    std::vector<std::thread> th;
    for (size_t k = 0; k < nth; ++k)
        th.emplace_back(check, pairs.size() * k / nth, pairs.size() * (k + 1) / nth);
    for (auto& x : th) x.join();
    if (!same.load()) return;
    // owners: each pair goes to the endpoint with fewer owned blocks so far
    std::vector<int> owned(nc, 0);
    std::vector<std::vector<std::pair<int64_t, int>>> own(nc);   // (near index of (owner, other), slot)
    std::vector<std::vector<int>> inc(nc);                        // slots landing in a leaf
    for (size_t q = 0; q < pairs.size(); ++q) {
        const Pair& pr = pairs[q];
        const bool to_t = owned[pr.t] <= owned[pr.s];
        const int ow = to_t ? pr.t : pr.s, ot = to_t ? pr.s : pr.t;
        owned[ow]++;
        own[ow].push_back({to_t ? pr.it : pr.is, int(q)});
        inc[ot].push_back(int(q));
    }
    std::vector<int> leaves;
    for (int c = 0; c < nc; ++c)
        if (d->nchild[c] == 0) leaves.push_back(c);
    std::stable_sort(leaves.begin(), leaves.end(), [&](int a, int b) { return owned[a] > owned[b]; });
    P.sym_leaf = leaves;
    P.sym_ptr.assign(1, 0);
    P.sym_in_ptr.assign(1, 0);
    for (int t : leaves) {
        for (int64_t i = nfirst[t]; i < nfirst[t] + ncount[t]; ++i)   // the diagonal block first
            if (d->near_s[i] == t) {
                P.sym_sbeg.push_back(int(d->begin[t]));
                P.sym_ssize.push_back(size(t));
                P.sym_off.push_back(P.near_uoff[i]);
                P.sym_pslot.push_back(-1);
            }
        for (auto& o : own[t]) {
            const int other = d->near_s[o.first];
            P.sym_sbeg.push_back(int(d->begin[other]));
            P.sym_ssize.push_back(size(other));
            P.sym_off.push_back(P.near_uoff[o.first]);
            P.sym_pslot.push_back(o.second);
        }
        P.sym_ptr.push_back(int(P.sym_off.size()));
        for (int q : inc[t]) P.sym_in_slot.push_back(q);
        P.sym_in_ptr.push_back(int(P.sym_in_slot.size()));
    }
    P.sym_pairs = int64_t(pairs.size());
    P.sym = true;
}

// Symmetric couplings: when every admissible pair (t, s) has its mirror (s, t) with
// S_st = S_ts^T bit for bit (checked here on host threads), the product can stream
// each unordered pair once.  The pair goes to t when (t < s) equals (t + s even),
// else to s: every cluster owns about half of its pairs wherever it sits in the
// numbering.  Each grouped block row is stored with its owned blocks first (the
// symmetric kernel streams that leading part; the full kernel the whole row, its
// gather index reordered alike).  Ranks above 4 * 16 rows per lane group are not
// handled (the mode is then not offered).  Needs P.row_cl / row_colptr / colsrc.
void plan_symmetric_couplings(const h2_host_desc* d, const std::vector<int64_t>& ffirst,
                              const std::vector<int64_t>& fcount, Plan& P) {
    const int nc = d->n_clusters;
    if (d->n_far == 0 || P.max_rank > 64) return;
    // each row's partners sorted, to find the mirror of a pair
    std::vector<std::pair<int, int64_t>> sorted(size_t(d->n_far));
    for (int t = 0; t < nc; ++t) {
        if (ffirst[t] < 0) continue;
        for (int64_t i = ffirst[t]; i < ffirst[t] + fcount[t]; ++i) sorted[size_t(i)] = {d->far_s[i], i};
        std::sort(sorted.begin() + ffirst[t], sorted.begin() + ffirst[t] + fcount[t]);
    }
    std::vector<int64_t> mirror(size_t(d->n_far), -1);
    for (int64_t i = 0; i < d->n_far; ++i) {
        const int t = d->far_t[i], s = d->far_s[i];
        if (ffirst[s] < 0) return;
        auto b = sorted.begin() + ffirst[s], e = b + fcount[s];
        auto it = std::lower_bound(b, e, std::pair<int, int64_t>(t, -1));
        if (it == e || it->first != t) return;
        mirror[size_t(i)] = it->second;
    }
    std::atomic<bool> same(true);
    auto check = [&](int64_t a, int64_t b) {
        for (int64_t i = a; i < b && same.load(std::memory_order_relaxed); ++i) {
            const int t = d->far_t[i], s = d->far_s[i];
            if (t >= s) continue;
            const int kt = d->rank[t], ks = d->rank[s];
            const double* sts = d->coupling + 2 * d->far_off[i];                 // kt x ks, column major
            const double* sst = d->coupling + 2 * d->far_off[mirror[size_t(i)]];  // ks x kt, column major
            for (int c = 0; c < ks; ++c)
                for (int r = 0; r < kt; ++r)
                    if (std::memcmp(sts + 2 * (int64_t(c) * kt + r), sst + 2 * (int64_t(r) * ks + c), 16) != 0) {
                        same.store(false);
                        return;
                    }
        }
    };
    const int64_t nth = std::max<int64_t>(1, std::min<int64_t>(8, d->n_far / 65536 + 1));
    std::vector<std::thread> th;
    for (int64_t k = 0; k < nth; ++k) th.emplace_back(check, d->n_far * k / nth, d->n_far * (k + 1) / nth);
    for (auto& x : th) x.join();
    if (!same.load()) return;
    auto owner = [](int t, int s) { return ((t < s) == (((t + s) & 1) == 0)) ? t : s; };
    const size_t nrow = P.row_cl.size();
    std::vector<int> slot_of(nc, -1);
    for (size_t q = 0; q < nrow; ++q) slot_of[P.row_cl[q]] = int(q);
    std::vector<std::vector<int>> recv(nrow);
    std::vector<int> row_nown(nrow, 0), row_pbase(nrow, 0), colsrc(P.colsrc);
    std::vector<int64_t> dev_off(size_t(d->n_far), 0);
    int64_t pcols = 0, elems = 0;
    for (size_t q = 0; q < nrow; ++q) {
        const int t = P.row_cl[q], kt = d->rank[t];
        row_pbase[q] = int(pcols);
        if (ffirst[t] < 0) continue;
        int col = 0;
        int64_t pos = P.row_colptr[q];
        for (int pass = 0; pass < 2; ++pass)            // owned blocks first, then the others
            for (int64_t i = ffirst[t]; i < ffirst[t] + fcount[t]; ++i) {
                const int s = d->far_s[i], ks = d->rank[s];
                const bool own = owner(t, s) == t;
                if (own != (pass == 0)) continue;
                dev_off[size_t(i)] = P.row_off[q] + int64_t(col) * kt;
                for (int b = 0; b < ks; ++b) colsrc[size_t(pos++)] = P.cl_coef[s] + b;
                if (own) {
                    recv[size_t(slot_of[s])].push_back(int(pcols + col));
                    elems += int64_t(kt) * ks;
                    row_nown[q] += ks;
                }
                col += ks;
            }
        pcols += row_nown[q];
        if (pcols >= (int64_t(1) << 31) / kNcomp) return;
    }
    P.row_nown = std::move(row_nown);
    P.row_pbase = std::move(row_pbase);
    P.colsrc = std::move(colsrc);
    P.coup_dev_off = std::move(dev_off);
    P.csym_elems = elems;
    P.csym_cols = pcols;
    P.crecv_ptr.assign(1, 0);
    for (size_t q = 0; q < nrow; ++q) {
        for (int p : recv[q]) P.crecv_p.push_back(p);
        P.crecv_ptr.push_back(int(P.crecv_p.size()));
    }
    P.csym = true;
}

// Tiles for the tiled near field: kTileLeaves leaves consecutive in tree order (the
// tree's leaves follow its spatial bisection, so a tile is a compact brick) and, per
// tile, one step per stored block that any of its leaves uses (a second step where a
// leaf uses the same stored block twice), in ascending storage order.
static void plan_near_tiles(const h2_host_desc* d, const std::vector<int64_t>& nfirst,
                            const std::vector<int64_t>& ncount, Plan& P) {
    P.tile_ptr.clear(); P.tile_leaf.clear(); P.step_shape.clear(); P.step_src.clear(); P.step_off.clear();
    P.tile_pairs = 0;
    if (!P.near_dedup) return;
    std::vector<int> leaves;
    for (int c = 0; c < d->n_clusters; ++c)
        if (d->nchild[c] == 0) leaves.push_back(c);
    std::stable_sort(leaves.begin(), leaves.end(), [&](int a, int b) { return d->begin[a] < d->begin[b]; });
    P.tile_ptr.push_back(0);
    for (size_t t0 = 0; t0 < leaves.size(); t0 += kTileLeaves) {
        // (stored offset, rows, columns) -> per slot, the sources' tree positions
        std::map<std::tuple<int64_t, int, int>, std::vector<std::vector<int>>> steps;
        for (int j = 0; j < kTileLeaves; ++j) {
            const int t = t0 + j < leaves.size() ? leaves[t0 + j] : -1;
            P.tile_leaf.push_back(t);
            if (t < 0) continue;
            const int nt = int(d->end[t] - d->begin[t]);
            for (int64_t i = nfirst[t]; i < nfirst[t] + ncount[t]; ++i) {
                const int s = d->near_s[i];
                auto& v = steps[std::make_tuple(P.near_uoff[i], nt, int(d->end[s] - d->begin[s]))];
                if (v.empty()) v.resize(kTileLeaves);
                v[j].push_back(int(d->begin[s]));
                P.tile_pairs++;
            }
        }
        for (auto& kv : steps) {
            size_t reps = 0;
            for (auto& v : kv.second) reps = std::max(reps, v.size());
            for (size_t r = 0; r < reps; ++r) {
                P.step_off.push_back(std::get<0>(kv.first));
                P.step_shape.push_back(std::get<1>(kv.first) | (std::get<2>(kv.first) << 16));
                for (int j = 0; j < kTileLeaves; ++j)
                    P.step_src.push_back(r < kv.second[j].size() ? kv.second[j][r] : -1);
            }
        }
        P.tile_ptr.push_back(int(P.step_off.size()));
    }
}

h2_status make_plan(const h2_host_desc* d, const h2_build_opts* o, Plan& P) {
    h2_status st = validate(d);
    if (st != H2_OK) return st;
    if (!o) return fail(H2_ERR_INVALID_ARG, "null build options");
    if (o->max_rhs < 1) return fail(H2_ERR_INVALID_ARG, "max_rhs must be >= 1");
    if (o->tiers & ~7) return fail(H2_ERR_INVALID_ARG, "unknown tier bits 0x%x", o->tiers);
    if (o->flags & ~H2_BUILD_KEEP_ALL_NEAR) return fail(H2_ERR_INVALID_ARG, "unknown build flags 0x%x", o->flags);
    P.tiers = o->tiers | 1;
    plan_near_dedup(d, (o->flags & H2_BUILD_KEEP_ALL_NEAR) == 0, P);
    const int nc = d->n_clusters;
    const int64_t n = d->n_vox;
    P.perm.assign(n, 0);
    for (int64_t p = 0; p < n; ++p) P.perm[p] = int(d->perm[p]);
    P.cl_rank.assign(d->rank, d->rank + nc);
    P.cl_coef.resize(nc);
    P.cl_begin.resize(nc);
    P.cl_size.resize(nc);
    P.cl_parent.assign(d->parent, d->parent + nc);
    P.cl_first_child.assign(d->first_child, d->first_child + nc);
    P.cl_nchild.assign(d->nchild, d->nchild + nc);
    P.cl_toff.assign(nc, -1);
    P.cl_boff.assign(nc, -1);
    int64_t coef = 0;
    for (int c = 0; c < nc; ++c) {
        P.cl_coef[c] = int(coef);
        coef += d->rank[c];
        P.cl_begin[c] = int(d->begin[c]);
        P.cl_size[c] = int(d->end[c] - d->begin[c]);
        P.depth = std::max(P.depth, int(d->level[c]));
        P.max_rank = std::max(P.max_rank, d->rank[c]);
        if (c > 0 && d->rank[c] > 0 && d->rank[d->parent[c]] > 0) P.cl_toff[c] = d->transfer_off[c];
        if (d->nchild[c] == 0 && d->rank[c] > 0) P.cl_boff[c] = d->basis_off[c];
    }
    if (coef >= (int64_t(1) << 31)) return fail(H2_ERR_BAD_DESC, "sum of ranks too large");
    P.coef_rows = int(coef);

    // leaves in launch order: most near blocks first
    std::vector<int> leaves;
    for (int c = 0; c < nc; ++c)
        if (d->nchild[c] == 0) {
            leaves.push_back(c);
            P.min_leaf_rank = std::min(P.min_leaf_rank, d->rank[c]);
        }
    std::vector<int64_t> nfirst(nc, 0), ncount(nc, 0);
    for (int64_t i = 0; i < d->n_near; ++i) {
        int t = d->near_t[i];
        if (ncount[t] == 0) nfirst[t] = i;
        ncount[t]++;
    }
    std::stable_sort(leaves.begin(), leaves.end(), [&](int a, int b) { return ncount[a] > ncount[b]; });
    P.leaf_id = leaves;
    // passes over the stored-once blocks: distinct blocks by use count, dealt in turn
    // to the passes (which evens out both their bytes and their work)
    std::map<int64_t, int> pass_of;                  // stored offset -> pass
    if (P.near_dedup) {
        const int64_t bytes = 16 * P.near_stored_len;
        P.near_passes = int(std::min<int64_t>(8, std::max<int64_t>(1, (bytes + kNearPassBytes - 1) / kNearPassBytes)));
        std::map<int64_t, int64_t> uses;
        for (int64_t i = 0; i < d->n_near; ++i) uses[P.near_uoff[i]]++;
        std::vector<std::pair<int64_t, int64_t>> order(uses.begin(), uses.end());
        std::stable_sort(order.begin(), order.end(), [](const auto& a, const auto& b) { return a.second > b.second; });
        for (size_t k = 0; k < order.size(); ++k) pass_of[order[k].first] = int(k % P.near_passes);
    }
    const int np = P.near_passes;
    P.near_ptr.assign(1, 0);
    P.near_pass_ptr.clear();
    for (int t : leaves) {
        for (int p = 0; p < np; ++p) {
            P.near_pass_ptr.push_back(int(P.near_off.size()));
            for (int64_t i = nfirst[t]; i < nfirst[t] + ncount[t]; ++i) {
                if (np > 1 && pass_of[P.near_uoff[i]] != p) continue;
                int s = d->near_s[i];
                P.near_sbeg.push_back(int(d->begin[s]));
                P.near_ssize.push_back(int(d->end[s] - d->begin[s]));
                P.near_off.push_back(P.near_uoff[i]);
            }
        }
        P.near_pass_ptr.push_back(int(P.near_off.size()));
        if (P.near_off.size() >= (size_t(1) << 31)) return fail(H2_ERR_BAD_DESC, "too many near blocks");
        P.near_ptr.push_back(int(P.near_off.size()));
    }

    plan_symmetric_near(d, nfirst, ncount, P);
    plan_near_tiles(d, nfirst, ncount, P);

    // leaves in cluster order with their diagonal near block (per-leaf preconditioners)
    for (int c = 0; c < nc; ++c) {
        if (d->nchild[c] != 0) continue;
        const int n = int(d->end[c] - d->begin[c]);
        int64_t diag = -1;
        for (int64_t i = nfirst[c]; i < nfirst[c] + ncount[c]; ++i)
            if (d->near_s[i] == c) diag = P.near_uoff[i];
        if (diag < 0) return fail(H2_ERR_BAD_DESC, "leaf %d has no diagonal near block", c);
        P.lc_beg.push_back(int(d->begin[c]));
        P.lc_size.push_back(n);
        P.lc_diag.push_back(diag);
        P.lc_inv.push_back(P.lc_inv_elems);
        P.lc_inv_elems += 2 * int64_t(n) * n;
        P.lc_max = std::max(P.lc_max, n);
    }

    // coupling rows: every cluster with rank > 0 (rows without blocks produce zeros)
    std::vector<int64_t> ffirst(nc, -1), fcount(nc, 0), fcols(nc, 0);
    for (int64_t i = 0; i < d->n_far; ++i) {
        int t = d->far_t[i];
        if (ffirst[t] < 0) ffirst[t] = i;
        fcount[t]++;
        fcols[t] += d->rank[d->far_s[i]];
    }
    std::vector<int> rows;
    for (int c = 0; c < nc; ++c)
        if (d->rank[c] > 0) rows.push_back(c);
    std::stable_sort(rows.begin(), rows.end(),
                     [&](int a, int b) { return fcols[a] * d->rank[a] > fcols[b] * d->rank[b]; });
    for (int t : rows) {
        P.row_cl.push_back(t);
        P.row_ncols.push_back(int(fcols[t]));
        P.row_colptr.push_back(int(P.colsrc.size()));
        P.row_off.push_back(ffirst[t] >= 0 ? d->far_off[ffirst[t]] : 0);
        for (int64_t i = ffirst[t]; ffirst[t] >= 0 && i < ffirst[t] + fcount[t]; ++i) {
            int s = d->far_s[i];
            for (int b = 0; b < d->rank[s]; ++b) P.colsrc.push_back(P.cl_coef[s] + b);
        }
        if (P.colsrc.size() >= (size_t(1) << 31)) return fail(H2_ERR_BAD_DESC, "too many coupling columns");
    }
    plan_symmetric_couplings(d, ffirst, fcount, P);

    // level lists: upward (deepest parents first), downward (top children first)
    for (int l = P.depth - 1; l >= 0; --l) {
        int b = int(P.up_list.size());
        for (int c = 0; c < nc; ++c)
            if (d->level[c] == l && d->nchild[c] > 0 && d->rank[c] > 0) P.up_list.push_back(c);
        P.lv.up_begin[P.lv.n_up] = b;
        P.lv.up_count[P.lv.n_up] = int(P.up_list.size()) - b;
        P.lv.n_up++;
    }
    for (int l = 1; l <= P.depth; ++l) {
        int b = int(P.down_list.size());
        for (int c = 0; c < nc; ++c)
            if (d->level[c] == l && P.cl_toff[c] >= 0) P.down_list.push_back(c);
        P.lv.down_begin[P.lv.n_down] = b;
        P.lv.down_count[P.lv.n_down] = int(P.down_list.size()) - b;
        P.lv.n_down++;
    }

    // device layout
    Layout& L = P.lay;
    auto ints = [](size_t k) { return std::max<size_t>(k, 1) * sizeof(int); };
    auto i64s = [](size_t k) { return std::max<size_t>(k, 1) * sizeof(int64_t); };
    P.o_perm = L.add(ints(n));
    P.o_chi = L.add(n * 16);
    for (int q = 0; q < 7; ++q) P.o_cl[q] = L.add(ints(nc));
    P.o_toff = L.add(i64s(nc));
    P.o_boff = L.add(i64s(nc));
    P.o_leaf = L.add(ints(P.leaf_id.size()));
    P.o_nptr = L.add(ints(P.near_ptr.size()));
    P.o_nsb = L.add(ints(P.near_sbeg.size()));
    P.o_nss = L.add(ints(P.near_ssize.size()));
    P.o_noff = L.add(i64s(P.near_off.size()));
    P.o_npass = L.add(ints(P.near_pass_ptr.size()));

    if (!P.tile_ptr.empty()) {
        const std::vector<int>* tv[4] = {&P.tile_ptr, &P.tile_leaf, &P.step_shape, &P.step_src};
        for (int q = 0; q < 4; ++q) P.o_tile[q] = L.add(ints(tv[q]->size()));
        P.o_stepoff = L.add(i64s(P.step_off.size()));
        P.o_tpart1 = L.add(size_t(n) * kNcomp * 16);
    }
    P.o_tzero = L.add(size_t(kMaxLeaf) * kNcomp * 16);
    if (P.near_passes > 1 || !P.tile_ptr.empty()) P.o_ypart = L.add(size_t(n) * kNcomp * 16);
    P.o_rowcl = L.add(ints(P.row_cl.size()));
    P.o_rownc = L.add(ints(P.row_ncols.size()));
    P.o_rowcp = L.add(ints(P.row_colptr.size()));
    P.o_colsrc = L.add(ints(P.colsrc.size()));
    P.o_rowoff = L.add(i64s(P.row_off.size()));
    if (P.csym) {
        const std::vector<int>* cv[4] = {&P.row_nown, &P.row_pbase, &P.crecv_ptr, &P.crecv_p};
        for (int q = 0; q < 4; ++q) P.o_csym[q] = L.add(ints(cv[q]->size()));
        P.o_cpart = L.add(size_t(std::max<int64_t>(P.csym_cols, 1)) * kNcomp * 16);
    }
    P.o_up = L.add(ints(P.up_list.size()));
    P.o_lbeg = L.add(ints(P.lc_beg.size()));
    P.o_lsize = L.add(ints(P.lc_size.size()));
    P.o_ldiag = L.add(i64s(P.lc_diag.size()));
    P.o_linv = L.add(i64s(P.lc_inv.size()));
    P.o_down = L.add(ints(P.down_list.size()));
    if (P.sym) {
        const std::vector<int>* sv[7] = {&P.sym_leaf, &P.sym_ptr, &P.sym_sbeg, &P.sym_ssize, &P.sym_pslot,
                                         &P.sym_in_ptr, &P.sym_in_slot};
        for (int q = 0; q < 7; ++q) P.o_sym[q] = L.add(ints(sv[q]->size()));
        P.o_symoff = L.add(i64s(P.sym_off.size()));
        P.o_sympart = L.add(size_t(std::max<int64_t>(P.sym_pairs, 1)) * kMaxLeaf * kNcomp * 16);
        P.o_symrows = L.add(size_t(n) * kNcomp * 16);
    }
    const int64_t lens[4] = {d->near_len, d->coupling_len, d->basis_len, d->transfer_len};
    for (int tier = 0; tier < 3; ++tier)
        for (int q = 0; q < 4; ++q) P.o_data[tier][q] = 0;
    const int64_t held[4] = {P.near_stored_len, lens[1], lens[2], lens[3]};
    for (int q = 0; q < 4; ++q) P.o_data[0][q] = L.add(std::max<int64_t>(held[q], 1) * 16);
    if (P.tiers & 2)
        for (int q = 0; q < 4; ++q) P.o_data[1][q] = L.add(std::max<int64_t>(held[q], 1) * 8);
    if (P.tiers & 4) {
        P.batch = new BatchHost();
        BatchHost& B = *P.batch;
        h2_status bs = plan_batch(d, o->max_rhs, P.near_uoff.data(), P.csym ? P.coup_dev_off.data() : nullptr, B);
        if (bs != H2_OK) return fail(bs, "batched tier needs ranks <= 64 and fewer than 2^31 padded rows");
        const size_t cols = size_t(B.max_cols);
        P.o_arena = L.add(size_t(std::max<int64_t>(B.arena_elems, 1)) * 2);
        P.o_ub = L.add(4 * size_t(B.urows) * cols * 2);
        P.o_xb = L.add(4 * size_t(B.crows) * cols * 2);
        P.o_yhb = L.add(4 * size_t(B.crows) * cols * 2);
        P.o_xf = L.add(2 * size_t(B.crows) * cols * 4);
        P.o_yhf = L.add(2 * size_t(B.crows) * cols * 4);
        P.o_yf = L.add(2 * size_t(B.urows) * cols * 4);
        P.o_prow = L.add(size_t(n) * 4);
        P.o_jobs = L.add(std::max<size_t>(B.jobs.size(), 1) * sizeof(PackJob));
        P.group_bytes = group_need_batch(&B);
        P.o_group = L.add(P.group_bytes);
    }
    const size_t cols = size_t(o->max_rhs >= 2 ? kMrCols : kNcomp);   // multi-RHS passes need kMrCols
    P.vec_cols = int(cols);
    P.o_U = L.add(size_t(n) * cols * 16);
    P.o_X = L.add(size_t(std::max(P.coef_rows, 1)) * cols * 16);
    P.o_Y = L.add(size_t(std::max(P.coef_rows, 1)) * cols * 16);
    P.aux_bytes = aux_scratch_bytes(n, P.coef_rows);
    P.o_aux = L.add(P.aux_bytes);
    return H2_OK;
}

}  // namespace

// Live handles: a destroyed or foreign pointer is rejected before it is read.
static std::mutex g_handles_mu;
static std::set<h2_handle> g_handles;

static bool handle_ok(h2_handle h) {
    if (h == nullptr) return false;
    std::lock_guard<std::mutex> lk(g_handles_mu);
    return g_handles.count(h) != 0 && h->magic == kHandleMagic;
}

extern "C" {

const char* h2_last_error(void) { return g_last_error.c_str(); }

h2_status h2_plan_from_host(const h2_host_desc* d, const h2_build_opts* o, size_t* dev_bytes) {
    if (!dev_bytes) return fail(H2_ERR_INVALID_ARG, "null dev_bytes");
    Plan P;
    h2_status st = make_plan(d, o, P);
    if (st != H2_OK) return st;
    *dev_bytes = P.lay.total + 256;
    return H2_OK;
}

h2_status h2_build_from_host(const h2_host_desc* d, const h2_build_opts* o, void* dev_buffer, size_t dev_bytes,
                             void* stream, h2_handle* out) {
    if (!out) return fail(H2_ERR_INVALID_ARG, "null output handle pointer");
    *out = nullptr;
    if (!dev_buffer) return fail(H2_ERR_INVALID_ARG, "null device buffer");
    Plan P;
    h2_status st = make_plan(d, o, P);
    if (st != H2_OK) return st;
    uintptr_t b = (reinterpret_cast<uintptr_t>(dev_buffer) + 255) & ~uintptr_t(255);
    size_t lost = b - reinterpret_cast<uintptr_t>(dev_buffer);
    if (dev_bytes < P.lay.total + lost) return fail(H2_ERR_OOM, "device buffer of %zu bytes, %zu needed", dev_bytes, P.lay.total + lost);
    char* base = reinterpret_cast<char*>(b);
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    auto put = [&](size_t off, const void* src, size_t bytes) -> hipError_t {
        if (bytes == 0) return hipSuccess;
        return hipMemcpyAsync(base + off, src, bytes, hipMemcpyHostToDevice, s);
    };
    std::vector<hipError_t> errs;
    const int nc = d->n_clusters;
    errs.push_back(put(P.o_perm, P.perm.data(), P.perm.size() * 4));
    errs.push_back(put(P.o_chi, d->chi, size_t(d->n_vox) * 16));
    const std::vector<int>* cl[7] = {&P.cl_rank, &P.cl_coef, &P.cl_begin, &P.cl_size, &P.cl_parent, &P.cl_first_child, &P.cl_nchild};
    for (int q = 0; q < 7; ++q) errs.push_back(put(P.o_cl[q], cl[q]->data(), size_t(nc) * 4));
    errs.push_back(put(P.o_toff, P.cl_toff.data(), size_t(nc) * 8));
    errs.push_back(put(P.o_boff, P.cl_boff.data(), size_t(nc) * 8));
    errs.push_back(put(P.o_leaf, P.leaf_id.data(), P.leaf_id.size() * 4));
    errs.push_back(put(P.o_nptr, P.near_ptr.data(), P.near_ptr.size() * 4));
    errs.push_back(put(P.o_nsb, P.near_sbeg.data(), P.near_sbeg.size() * 4));
    errs.push_back(put(P.o_nss, P.near_ssize.data(), P.near_ssize.size() * 4));
    errs.push_back(put(P.o_noff, P.near_off.data(), P.near_off.size() * 8));
    errs.push_back(put(P.o_npass, P.near_pass_ptr.data(), P.near_pass_ptr.size() * 4));
    if (!P.tile_ptr.empty()) {
        const std::vector<int>* tv[4] = {&P.tile_ptr, &P.tile_leaf, &P.step_shape, &P.step_src};
        for (int q = 0; q < 4; ++q) errs.push_back(put(P.o_tile[q], tv[q]->data(), tv[q]->size() * 4));
        errs.push_back(put(P.o_stepoff, P.step_off.data(), P.step_off.size() * 8));
    }
    const std::vector<double> zeros(size_t(kMaxLeaf) * kNcomp * 2, 0.0);
    errs.push_back(put(P.o_tzero, zeros.data(), zeros.size() * 8));

    errs.push_back(put(P.o_rowcl, P.row_cl.data(), P.row_cl.size() * 4));
    errs.push_back(put(P.o_rownc, P.row_ncols.data(), P.row_ncols.size() * 4));
    errs.push_back(put(P.o_rowcp, P.row_colptr.data(), P.row_colptr.size() * 4));
    errs.push_back(put(P.o_colsrc, P.colsrc.data(), P.colsrc.size() * 4));
    errs.push_back(put(P.o_rowoff, P.row_off.data(), P.row_off.size() * 8));
    if (P.csym) {
        const std::vector<int>* cv[4] = {&P.row_nown, &P.row_pbase, &P.crecv_ptr, &P.crecv_p};
        for (int q = 0; q < 4; ++q) errs.push_back(put(P.o_csym[q], cv[q]->data(), cv[q]->size() * 4));
    }
    errs.push_back(put(P.o_up, P.up_list.data(), P.up_list.size() * 4));
    errs.push_back(put(P.o_lbeg, P.lc_beg.data(), P.lc_beg.size() * 4));
    errs.push_back(put(P.o_lsize, P.lc_size.data(), P.lc_size.size() * 4));
    errs.push_back(put(P.o_ldiag, P.lc_diag.data(), P.lc_diag.size() * 8));
    errs.push_back(put(P.o_linv, P.lc_inv.data(), P.lc_inv.size() * 8));
    errs.push_back(put(P.o_down, P.down_list.data(), P.down_list.size() * 4));
    if (P.sym) {
        const std::vector<int>* sv[7] = {&P.sym_leaf, &P.sym_ptr, &P.sym_sbeg, &P.sym_ssize, &P.sym_pslot,
                                         &P.sym_in_ptr, &P.sym_in_slot};
        for (int q = 0; q < 7; ++q) errs.push_back(put(P.o_sym[q], sv[q]->data(), sv[q]->size() * 4));
        errs.push_back(put(P.o_symoff, P.sym_off.data(), P.sym_off.size() * 8));
    }
    const double* src[4] = {d->near_blocks, d->coupling, d->basis, d->transfer};
    const int64_t lens[4] = {P.near_stored_len, d->coupling_len, d->basis_len, d->transfer_len};
    std::vector<double> near_staged;        // the stored near blocks, gathered (identical blocks once)
    if (P.near_dedup) {
        near_staged.resize(size_t(2 * P.near_stored_len));
        for (int64_t i : P.near_src) {
            const int64_t n = (d->end[d->near_t[i]] - d->begin[d->near_t[i]]) * (d->end[d->near_s[i]] - d->begin[d->near_s[i]]);
            std::memcpy(near_staged.data() + 2 * P.near_uoff[i], d->near_blocks + 2 * d->near_off[i], size_t(n) * 16);
        }
        src[0] = near_staged.data();
    }
    std::vector<double> coup_staged;        // grouped rows with their owned blocks first
    if (P.csym) {
        coup_staged.resize(size_t(2 * d->coupling_len));
        auto fill = [&](int64_t a, int64_t b) {
            for (int64_t i = a; i < b; ++i) {
                const int64_t n = int64_t(d->rank[d->far_t[i]]) * d->rank[d->far_s[i]];
                std::memcpy(coup_staged.data() + 2 * P.coup_dev_off[size_t(i)], d->coupling + 2 * d->far_off[i],
                            size_t(n) * 16);
            }
        };
        const int64_t nth = std::max<int64_t>(1, std::min<int64_t>(8, d->n_far / 65536 + 1));
        std::vector<std::thread> th;
        for (int64_t k = 0; k < nth; ++k) th.emplace_back(fill, d->n_far * k / nth, d->n_far * (k + 1) / nth);
        for (auto& x : th) x.join();
        src[1] = coup_staged.data();
    }
    for (int q = 0; q < 4; ++q) errs.push_back(put(P.o_data[0][q], src[q], size_t(lens[q]) * 16));
    for (hipError_t e : errs)
        if (e != hipSuccess) {
            (void)hipStreamSynchronize(s);     // no copy may still read the host staging
            return fail(H2_ERR_DEVICE, "upload failed: %s", hipGetErrorString(e));
        }
    // lower-precision tiers converted on the device from the FP64 copy
    for (int q = 0; q < 4; ++q) {
        if (lens[q] == 0) continue;
        if (P.tiers & 2) {
            hipError_t e = launch_convert_fp32((const double2*)(base + P.o_data[0][q]), (float2*)(base + P.o_data[1][q]), lens[q], s);
            if (e != hipSuccess) {
                (void)hipStreamSynchronize(s);
                return fail(H2_ERR_DEVICE, "fp32 conversion failed: %s", hipGetErrorString(e));
            }
        }
    }
    hipError_t e = hipStreamSynchronize(s);       // also the last read of the near staging
    if (e != hipSuccess) return fail(H2_ERR_DEVICE, "build synchronisation failed: %s", hipGetErrorString(e));

    h2_handle h = new h2_handle_s();
    if (hipGetDevice(&h->device) != hipSuccess) h->device = -1;
    DevH2& D = h->dev;
    D.n_vox = int(d->n_vox);
    D.n_clusters = nc;
    D.n_leaves = int(P.leaf_id.size());
    D.coef_rows = P.coef_rows;
    D.n_rowcl = int(P.row_cl.size());
    D.coupling_mr_mfma = P.max_rank <= 64;
    D.depth = P.depth;
    D.k = d->k;
    D.volume = d->volume;
    D.sigma = d->sigma;
    D.perm = (const int*)(base + P.o_perm);
    D.chi = (const double2*)(base + P.o_chi);
    D.cl_rank = (const int*)(base + P.o_cl[0]);
    D.cl_coef = (const int*)(base + P.o_cl[1]);
    D.cl_begin = (const int*)(base + P.o_cl[2]);
    D.cl_size = (const int*)(base + P.o_cl[3]);
    D.cl_parent = (const int*)(base + P.o_cl[4]);
    D.cl_first_child = (const int*)(base + P.o_cl[5]);
    D.cl_nchild = (const int*)(base + P.o_cl[6]);
    D.cl_transfer_off = (const int64_t*)(base + P.o_toff);
    D.cl_basis_off = (const int64_t*)(base + P.o_boff);
    D.leaf_id = (const int*)(base + P.o_leaf);
    D.near_ptr = (const int*)(base + P.o_nptr);
    D.near_sbeg = (const int*)(base + P.o_nsb);
    D.near_ssize = (const int*)(base + P.o_nss);
    D.near_off = (const int64_t*)(base + P.o_noff);
    D.row_cl = (const int*)(base + P.o_rowcl);
    D.row_ncols = (const int*)(base + P.o_rownc);
    D.row_colptr = (const int*)(base + P.o_rowcp);
    D.colsrc = (const int*)(base + P.o_colsrc);
    D.row_off = (const int64_t*)(base + P.o_rowoff);
    if (P.csym) {
        D.coup_sym_ok = true;
        D.coup_sym = false;               // measured no faster than streaming every block
        D.row_nown = (const int*)(base + P.o_csym[0]);
        D.row_pbase = (const int*)(base + P.o_csym[1]);
        D.crecv_ptr = (const int*)(base + P.o_csym[2]);
        D.crecv_p = (const int*)(base + P.o_csym[3]);
        D.cpart = base + P.o_cpart;
    }
    D.up_list = (const int*)(base + P.o_up);
    D.leaves.n = int(P.lc_beg.size());
    D.leaves.beg = (const int*)(base + P.o_lbeg);
    D.leaves.size = (const int*)(base + P.o_lsize);
    D.leaves.diag = (const int64_t*)(base + P.o_ldiag);
    D.leaves.inv_off = (const int64_t*)(base + P.o_linv);
    D.leaves.inv_elems = P.lc_inv_elems;
    D.leaves.max_leaf = P.lc_max;
    D.down_list = (const int*)(base + P.o_down);
    D.near_cached = P.near_dedup;
    D.near_passes = P.near_passes;
    D.near_pass_ptr = (const int*)(base + P.o_npass);

    D.zero_block = base + P.o_tzero;
    D.near_ypart = P.near_passes > 1 || !P.tile_ptr.empty() ? base + P.o_ypart : nullptr;
    if (!P.tile_ptr.empty()) {
        D.near_tiles_ok = true;
        D.near_tiles = true;
        D.n_tiles = int(P.tile_ptr.size()) - 1;
        D.tile_ptr = (const int*)(base + P.o_tile[0]);
        D.tile_leaf = (const int*)(base + P.o_tile[1]);
        D.step_shape = (const int*)(base + P.o_tile[2]);
        D.step_src = (const int*)(base + P.o_tile[3]);
        D.step_off = (const int64_t*)(base + P.o_stepoff);
        D.tiles_full = std::all_of(P.step_shape.begin(), P.step_shape.end(),
                                   [](int sh) { return sh == (kMaxLeaf | (kMaxLeaf << 16)); });
        D.tile_part1 = base + P.o_tpart1;
    }
    if (P.near_passes > 1 || !P.tile_ptr.empty()) {   // side stream (default priority) for near work that needs only U
        hipStream_t side = nullptr;
        hipEvent_t ef = nullptr, ej = nullptr;
        if (hipStreamCreateWithFlags(&side, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&ef, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&ej, hipEventDisableTiming) == hipSuccess) {
            D.near_side = side;
            D.near_fork = ef;
            D.near_join = ej;
        } else {   // no overlap: the passes run in order on the product's stream
            if (side) (void)hipStreamDestroy(side);
            if (ef) (void)hipEventDestroy(ef);
            if (ej) (void)hipEventDestroy(ej);
            (void)hipGetLastError();
        }
    }
    if (P.sym) {
        D.near_sym_ok = true;
        // halving the block stream pays when the blocks come from HBM; blocks stored
        // once are read from the caches, where the one-sided full mode is faster
        D.near_sym = !P.near_dedup;
        D.sym_leaf = (const int*)(base + P.o_sym[0]);
        D.sym_ptr = (const int*)(base + P.o_sym[1]);
        D.sym_sbeg = (const int*)(base + P.o_sym[2]);
        D.sym_ssize = (const int*)(base + P.o_sym[3]);
        D.sym_pslot = (const int*)(base + P.o_sym[4]);
        D.sym_in_ptr = (const int*)(base + P.o_sym[5]);
        D.sym_in_slot = (const int*)(base + P.o_sym[6]);
        D.sym_off = (const int64_t*)(base + P.o_symoff);
        D.sym_part = base + P.o_sympart;
        D.sym_rows = base + P.o_symrows;
    }
    for (int tier = 0; tier < 3; ++tier) {
        D.has_tier[tier] = (P.tiers >> tier) & 1;
        if (!D.has_tier[tier] || tier == 2) continue;
        D.tier[tier].near = base + P.o_data[tier][0];
        D.tier[tier].coupling = base + P.o_data[tier][1];
        D.tier[tier].basis = base + P.o_data[tier][2];
        D.tier[tier].transfer = base + P.o_data[tier][3];
    }
    if (P.tiers & 4) {
        BatchHost* B = P.batch;
        P.batch = nullptr;
        h->batch = B;
        B->arena = (uint16_t*)(base + P.o_arena);
        B->Ub = (uint16_t*)(base + P.o_ub);
        B->Xb = (uint16_t*)(base + P.o_xb);
        B->Yhb = (uint16_t*)(base + P.o_yhb);
        B->Xf = (float*)(base + P.o_xf);
        B->Yhf = (float*)(base + P.o_yhf);
        B->Yf = (float*)(base + P.o_yf);
        B->prow_dev = (int*)(base + P.o_prow);
        const size_t cols = size_t(B->max_cols);
        hipError_t e2 = hipMemcpyAsync(B->prow_dev, B->prow.data(), B->prow.size() * 4, hipMemcpyHostToDevice, s);
        if (e2 == hipSuccess && !B->jobs.empty())
            e2 = hipMemcpyAsync(base + P.o_jobs, B->jobs.data(), B->jobs.size() * sizeof(PackJob), hipMemcpyHostToDevice, s);
        // bf16 vector planes start at zero (their padding rows stay zero)
        if (e2 == hipSuccess) e2 = launch_fill_u16(B->Ub, 4 * int64_t(B->urows) * int64_t(cols), s);
        if (e2 == hipSuccess) e2 = launch_fill_u16(B->Xb, 4 * int64_t(B->crows) * int64_t(cols), s);
        if (e2 == hipSuccess) e2 = launch_fill_u16(B->Yhb, 4 * int64_t(B->crows) * int64_t(cols), s);
        const double2* srcs[4] = {(const double2*)(base + P.o_data[0][0]), (const double2*)(base + P.o_data[0][1]),
                                  (const double2*)(base + P.o_data[0][2]), (const double2*)(base + P.o_data[0][3])};
        if (e2 == hipSuccess)
            e2 = launch_pack((const PackJob*)(base + P.o_jobs), int(B->jobs.size()), srcs, B->arena, s);
        if (e2 == hipSuccess) e2 = hipStreamSynchronize(s);
        B->jobs.clear();
        B->jobs.shrink_to_fit();
        if (e2 != hipSuccess) {
            delete h;
            return fail(H2_ERR_DEVICE, "batched tier packing failed: %s", hipGetErrorString(e2));
        }
    }
    D.U = base + P.o_U;
    D.vec_cols = P.vec_cols;
    D.Xh = base + P.o_X;
    D.Yh = base + P.o_Y;
    h->aux = base + P.o_aux;
    h->aux_bytes = P.aux_bytes;
    h->lv = P.lv;
    h->base = base;
    h->bytes = P.lay.total;
    h->tiers = P.tiers;
    h2_stats_t& S = h->stats;
    S.n_vox = d->n_vox;
    S.n_clusters = nc;
    S.n_leaves = D.n_leaves;
    S.n_far = d->n_far;
    S.n_near = d->n_near;
    S.depth = P.depth;
    S.near_elems = d->near_len;
    S.near_stored_elems = P.near_stored_len;
    S.near_unique = P.near_dedup ? int64_t(P.near_src.size()) : d->n_near;
    S.near_passes = D.near_passes;
    S.near_tiles = D.n_tiles;
    S.near_tile_steps = int64_t(P.step_off.size());
    S.coupling_owned_elems = P.csym ? P.csym_elems : 0;
    S.coupling_owned_cols = P.csym ? P.csym_cols : 0;
    S.coupling_elems = d->coupling_len;
    S.basis_elems = d->basis_len;
    S.transfer_elems = d->transfer_len;
    S.coef_rows = P.coef_rows;
    S.max_rank = P.max_rank;
    S.min_leaf_rank = P.min_leaf_rank;
    S.dev_bytes = int64_t(P.lay.total + 256);
    const double blocks = double(d->near_len + d->coupling_len + d->basis_len + d->transfer_len);
    S.bytes_fp64 = (blocks + 2.0 * double(d->n_vox) * kNcomp) * 16.0;
    S.flops_fp64 = 8.0 * kNcomp * (double(d->near_len) + double(d->coupling_len) + 2.0 * double(d->basis_len) +
                                   2.0 * double(d->transfer_len));
    {
        std::lock_guard<std::mutex> lk(g_handles_mu);
        g_handles.insert(h);
    }
    if (h->batch) {
        h2_status gs = group_create(&h, 1, base + P.o_group, P.group_bytes, s, &h->self_group);
        if (gs != H2_OK) {
            h2_destroy(h);
            return gs;
        }
    }
    *out = h;
    return H2_OK;
}

h2_status h2_matvec(h2_handle h, h2_op op, h2_precision p, const void* x, void* y, int64_t n_rhs, int64_t ld,
                    void* stream) {
    if (!handle_ok(h)) return fail(H2_ERR_BAD_HANDLE, "invalid handle");
    if (op != H2_OP_G && op != H2_OP_Z) return fail(H2_ERR_INVALID_ARG, "unknown op %d", int(op));
    if (p < H2_FP64 || p > H2_BF16X3) return fail(H2_ERR_INVALID_ARG, "unknown precision %d", int(p));
    if (!h->dev.has_tier[p]) return fail(H2_ERR_INVALID_ARG, "precision tier %d was not built", int(p));
    if (!x || !y) return fail(H2_ERR_INVALID_ARG, "null vector");
    const int64_t N = int64_t(h->dev.n_vox) * kNcomp;
    if (n_rhs < 1) return fail(H2_ERR_INVALID_ARG, "n_rhs must be >= 1");
    if (ld < N) return fail(H2_ERR_INVALID_ARG, "ld (%lld) < N (%lld)", (long long)ld, (long long)N);
    const size_t esz = (p == H2_FP64) ? 16 : 8;
    if ((reinterpret_cast<uintptr_t>(x) | reinterpret_cast<uintptr_t>(y)) % esz)
        return fail(H2_ERR_INVALID_ARG, "misaligned vector");
    const char* xb = (const char*)x;
    const char* yb = (const char*)y;
    const size_t span = size_t((n_rhs - 1) * ld + N) * esz;
    if (xb < yb + span && yb < xb + span) return fail(H2_ERR_INVALID_ARG, "x and y overlap");
    if (p == H2_BF16X3) {
        const void* xs[1] = {x};
        void* ys[1] = {y};
        const int64_t nr[1] = {n_rhs}, lds[1] = {ld};
        return group_run(h->self_group, int(op), xs, ys, nr, lds, reinterpret_cast<hipStream_t>(stream));
    }
    hipError_t e = (n_rhs > 1 && !h->prof)
                       ? launch_matvec_multi(h->dev, h->lv, int(op), int(p), x, y, n_rhs, ld,
                                             reinterpret_cast<hipStream_t>(stream))
                       : launch_matvec(h->dev, h->lv, int(op), int(p), x, y, n_rhs, ld,
                                       reinterpret_cast<hipStream_t>(stream), h->prof);
    if (e != hipSuccess) return fail(H2_ERR_DEVICE, "matvec launch failed: %s", hipGetErrorString(e));
    return H2_OK;
}

h2_status h2_coupling_mode(h2_handle h, int32_t set, int32_t* mode, int32_t* available) {
    if (!handle_ok(h)) return fail(H2_ERR_BAD_HANDLE, "invalid handle");
    if (set < -1 || set > 1) return fail(H2_ERR_INVALID_ARG, "coupling mode must be -1, 0 or 1");
    if (set == 1 && !h->dev.coup_sym_ok)
        return fail(H2_ERR_INVALID_ARG, "the couplings are not symmetric: no symmetric coupling mode");
    if (set >= 0) h->dev.coup_sym = set == 1;
    if (mode) *mode = h->dev.coup_sym ? 1 : 0;
    if (available) *available = h->dev.coup_sym_ok ? 1 : 0;
    return H2_OK;
}

h2_status h2_near_mode(h2_handle h, int32_t set, int32_t* mode, int32_t* available) {
    if (!handle_ok(h)) return fail(H2_ERR_BAD_HANDLE, "invalid handle");
    if (set < -1 || set > 1) return fail(H2_ERR_INVALID_ARG, "near mode must be -1, 0 or 1");
    if (set == 1 && !h->dev.near_sym_ok)
        return fail(H2_ERR_INVALID_ARG, "the near blocks are not symmetric: no symmetric near mode");
    if (set >= 0) h->dev.near_sym = set == 1;
    if (mode) *mode = h->dev.near_sym ? 1 : 0;
    if (available) *available = h->dev.near_sym_ok ? 1 : 0;
    return H2_OK;
}

h2_status h2_near_tiles(h2_handle h, int32_t set, int32_t* on, int32_t* available) {
    if (!handle_ok(h)) return fail(H2_ERR_BAD_HANDLE, "invalid handle");
    if (set < -1 || set > 1) return fail(H2_ERR_INVALID_ARG, "near tiles setting must be -1, 0 or 1");
    if (set == 1 && !h->dev.near_tiles_ok)
        return fail(H2_ERR_INVALID_ARG, "near blocks are not stored once: no tiled near field");
    if (set >= 0) h->dev.near_tiles = set == 1;
    if (on) *on = h->dev.near_tiles ? 1 : 0;
    if (available) *available = h->dev.near_tiles_ok ? 1 : 0;
    return H2_OK;
}

h2_status h2_profile_enable(h2_handle h, int enable) {
    if (!handle_ok(h)) return fail(H2_ERR_BAD_HANDLE, "invalid handle");
    if (enable && !h->prof) h->prof = new EventProfiler();
    if (!enable && h->prof) {
        if (hipDeviceSynchronize() != hipSuccess) return fail(H2_ERR_DEVICE, "synchronisation failed");
        delete h->prof;
        h->prof = nullptr;
    }
    return H2_OK;
}

h2_status h2_profile_read(h2_handle h, h2_kernel_times* out) {
    if (!handle_ok(h)) return fail(H2_ERR_BAD_HANDLE, "invalid handle");
    if (!out) return fail(H2_ERR_INVALID_ARG, "null output");
    *out = h2_kernel_times{};
    if (!h->prof) return H2_OK;
    for (auto& r : h->prof->done) {
        if (hipEventSynchronize(r.b) != hipSuccess) return fail(H2_ERR_DEVICE, "event synchronisation failed");
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return fail(H2_ERR_DEVICE, "event timing failed");
        if (r.family >= 0 && r.family < H2_K_FAMILIES) {
            out->ms[r.family] += ms;
            out->launches[r.family] += 1;
        }
        h->prof->pool.push_back(r.a);
        h->prof->pool.push_back(r.b);
    }
    h->prof->done.clear();
    return H2_OK;
}

h2_status h2_stats(h2_handle h, h2_stats_t* out) {
    if (!handle_ok(h)) return fail(H2_ERR_BAD_HANDLE, "invalid handle");
    if (!out) return fail(H2_ERR_INVALID_ARG, "null stats");
    *out = h->stats;
    return H2_OK;
}

void h2_destroy(h2_handle h) {
    if (!handle_ok(h)) return;
    {
        std::lock_guard<std::mutex> lk(g_handles_mu);
        g_handles.erase(h);
    }
    h->magic = 0;
    delete h;
}

}  // extern "C"

// accessors used by the solver translation unit
namespace h2 {
const DevH2* handle_dev(h2_handle h) { return handle_ok(h) ? &h->dev : nullptr; }
const LevelLaunch* handle_levels(h2_handle h) { return handle_ok(h) ? &h->lv : nullptr; }
void* handle_aux(h2_handle h, size_t* bytes) {
    if (!handle_ok(h)) return nullptr;
    *bytes = h->aux_bytes;
    return h->aux;
}
bool handle_live(h2_handle h) { return handle_ok(h); }
h2_status handle_fail(h2_status st, const char* msg) {
    g_last_error = msg;
    return st;
}
}  // namespace h2
