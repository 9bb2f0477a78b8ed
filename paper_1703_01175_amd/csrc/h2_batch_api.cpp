// Host side of the batched BF16x3 tier: plan of the operand planes and phase
// lists of one representation, groups of representations run phase by phase
// in shared launches (captured in a HIP graph), and the tile autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/h2vie.h"
#include "h2_api_internal.h"
#include "h2_batch.h"

namespace h2 {

static inline int pad16(int v) { return (v + 15) & ~15; }

// ---------------------------------------------------------------- plan of one representation
h2_status plan_batch(const h2_host_desc* d, int max_rhs, const int64_t* near_off, const int64_t* coup_off,
                     BatchHost& B) {
    const int nc = d->n_clusters;
    for (int c = 0; c < nc; ++c)
        if (d->rank[c] > 64) return H2_ERR_BAD_DESC;      // row blocks of the block GEMM hold <= 64 rows
    B.max_cols = 3 * max_rhs;
    // padded rows of the coefficient planes, cluster order (levels are contiguous)
    std::vector<int64_t> crow(nc + 1, 0);
    for (int c = 0; c < nc; ++c) crow[c + 1] = crow[c] + pad16(d->rank[c]);
    B.crows = std::max<int64_t>(crow[nc], 16);
    // padded rows of the voxel planes: leaves in cluster order
    std::vector<int64_t> urow(nc, -1);
    int64_t u = 0;
    for (int c = 0; c < nc; ++c)
        if (d->nchild[c] == 0) {
            urow[c] = u;
            u += pad16(int(d->end[c] - d->begin[c]));
        }
    B.urows = u;
    B.prow.assign(d->n_vox, 0);
    for (int c = 0; c < nc; ++c)
        if (d->nchild[c] == 0)
            for (int64_t p = d->begin[c]; p < d->end[c]; ++p) B.prow[p] = int(urow[c] + (p - d->begin[c]));
    for (int64_t r : B.prow)
        if (r >= (int64_t(1) << 31)) return H2_ERR_BAD_DESC;

    int64_t arena = 0;
    bool too_big = false;   // the block GEMM stages at most 64 complex k and holds at most 64 rows per block
    auto add_job = [&](int which, int64_t src, int m, int k, int src_rows, int transpose) -> int64_t {
        too_big = too_big || m > 64 || k > 64;
        PackJob J{};
        J.src = src;
        J.dst = arena;
        J.m = m;
        J.k = k;
        J.mp = pad16(m);
        J.kp = pad16(k);
        J.src_rows = src_rows;
        J.transpose = transpose;
        J.which = which;
        B.jobs.push_back(J);
        const int64_t off = arena;
        arena += 4 * int64_t(J.mp) * J.kp;
        return off;
    };
    auto size = [&](int c) { return int(d->end[c] - d->begin[c]); };

    // leaf forward: X_t = V_t^T U_t
    for (int c = 0; c < nc; ++c)
        if (d->nchild[c] == 0 && d->rank[c] > 0) {
            const int n = size(c), k = d->rank[c];
            const int64_t a = add_job(2, d->basis_off[c], k, n, n, 1);
            B.leaf.owners.push_back({0, crow[c], pad16(k), int(B.leaf.terms.size()), 1, 0});
            B.leaf.terms.push_back({a, 0, urow[c], pad16(n)});
        }
    B.leaf.split_kind = 0;
    B.leaf.split_r0 = 0;
    B.leaf.split_rows = B.crows;
    // upward: X_p = sum_c T_c^T X_c, deepest parents first
    int depth = 0;
    for (int c = 0; c < nc; ++c) depth = std::max(depth, d->level[c]);
    for (int l = depth - 1; l >= 0; --l) {
        RelPhase ph;
        int64_t r0 = -1, r1 = -1;
        for (int p = 0; p < nc; ++p) {
            if (d->level[p] != l) continue;
            if (r0 < 0) r0 = crow[p];
            r1 = crow[p + 1];
            if (d->nchild[p] == 0 || d->rank[p] == 0) continue;
            RelOwner o{0, crow[p], pad16(d->rank[p]), int(ph.terms.size()), 0, 0};
            for (int ch = d->first_child[p]; ch < d->first_child[p] + d->nchild[p]; ++ch) {
                if (d->rank[ch] == 0) continue;
                const int kc = d->rank[ch], kp = d->rank[p];
                const int64_t a = add_job(3, d->transfer_off[ch], kp, kc, kc, 1);
                ph.terms.push_back({a, 1, crow[ch], pad16(kc)});
                o.nt++;
            }
            ph.owners.push_back(o);
        }
        ph.split_kind = 0;
        ph.split_r0 = std::max<int64_t>(r0, 0);
        ph.split_rows = std::max<int64_t>(r1 - r0, 0);
        B.up.push_back(ph);
    }
    // couplings: every cluster with rank > 0 (no terms -> zero output)
    {
        std::vector<int64_t> ffirst(nc, -1), fcount(nc, 0);
        for (int64_t i = 0; i < d->n_far; ++i) {
            const int t = d->far_t[i];
            if (ffirst[t] < 0) ffirst[t] = i;
            fcount[t]++;
        }
        for (int t = 0; t < nc; ++t) {
            if (d->rank[t] == 0) continue;
            RelOwner o{1, crow[t], pad16(d->rank[t]), int(B.coup.terms.size()), 0, 0};
            for (int64_t i = ffirst[t]; ffirst[t] >= 0 && i < ffirst[t] + fcount[t]; ++i) {
                const int s = d->far_s[i];
                const int64_t a = add_job(1, coup_off ? coup_off[i] : d->far_off[i], d->rank[t], d->rank[s], d->rank[t], 0);
                B.coup.terms.push_back({a, 1, crow[s], pad16(d->rank[s])});
                o.nt++;
            }
            B.coup.owners.push_back(o);
        }
        B.coup.split_kind = 1;
        B.coup.split_r0 = 0;
        B.coup.split_rows = B.crows;
    }
    // downward: Y_c += T_c Y_p, top children first
    for (int l = 1; l <= depth; ++l) {
        RelPhase ph;
        int64_t r0 = -1, r1 = -1;
        for (int c = 0; c < nc; ++c) {
            if (d->level[c] != l) continue;
            if (r0 < 0) r0 = crow[c];
            r1 = crow[c + 1];
            const int p = d->parent[c];
            if (d->rank[c] == 0 || d->rank[p] == 0) continue;
            const int64_t a = add_job(3, d->transfer_off[c], d->rank[c], d->rank[p], d->rank[c], 0);
            ph.owners.push_back({1, crow[c], pad16(d->rank[c]), int(ph.terms.size()), 1, 1});
            ph.terms.push_back({a, 2, crow[p], pad16(d->rank[p])});
        }
        ph.split_kind = 1;
        ph.split_r0 = std::max<int64_t>(r0, 0);
        ph.split_rows = std::max<int64_t>(r1 - r0, 0);
        B.down.push_back(ph);
    }
    // near field + leaf backward: y_t = sum_s G_ts U_s + V_t Y_t
    {
        std::map<std::pair<int64_t, std::pair<int, int>>, int64_t> packed_near;
        std::vector<int64_t> nfirst(nc, -1), ncount(nc, 0);
        for (int64_t i = 0; i < d->n_near; ++i) {
            const int t = d->near_t[i];
            if (nfirst[t] < 0) nfirst[t] = i;
            ncount[t]++;
        }
        std::vector<int> leaves;
        for (int c = 0; c < nc; ++c)
            if (d->nchild[c] == 0) leaves.push_back(c);
        std::stable_sort(leaves.begin(), leaves.end(), [&](int a, int b) { return ncount[a] > ncount[b]; });
        for (int t : leaves) {
            const int n = size(t);
            RelOwner o{2, urow[t], pad16(n), int(B.near.terms.size()), 0, 0};
            for (int64_t i = nfirst[t]; nfirst[t] >= 0 && i < nfirst[t] + ncount[t]; ++i) {
                const int s = d->near_s[i];
                // near blocks stored once (identical blocks) are packed once too
                auto key = std::make_pair(near_off[i], std::make_pair(n, size(s)));
                auto hit = packed_near.find(key);
                const int64_t a = hit != packed_near.end() ? hit->second : add_job(0, near_off[i], n, size(s), n, 0);
                packed_near.emplace(key, a);
                B.near.terms.push_back({a, 0, urow[s], pad16(size(s))});
                o.nt++;
            }
            if (d->rank[t] > 0) {
                const int64_t a = add_job(2, d->basis_off[t], n, d->rank[t], n, 0);
                B.near.terms.push_back({a, 2, crow[t], pad16(d->rank[t])});
                o.nt++;
            }
            B.near.owners.push_back(o);
        }
    }
    if (too_big) return H2_ERR_BAD_DESC;
    B.arena_elems = arena;
    return H2_OK;
}

// ---------------------------------------------------------------- groups
struct GroupMember {
    h2_handle h;
    BatchHost* B;
    int ncols = 0;              // columns of the current call
};

struct GroupDev {               // device arrays of one phase
    BOwner* owners = nullptr;
    BTerm* terms = nullptr;
    SplitSeg* splits = nullptr;
    int* split_cols = nullptr;
    int2* tasks = nullptr;
    int* owner_cols = nullptr;
    int n_owners = 0, n_terms = 0, n_splits = 0, max_tasks = 0, n_tasks = 0;
    int64_t max_split_elems = 0;
};

}  // namespace h2

struct h2_group_s {
    uint32_t magic = 0x48324752u;  // "H2GR"
    std::vector<h2::GroupMember> members;
    std::vector<h2::GPhase> host;   // phase order: leaf, up..., coup, down..., near
    std::vector<h2::GroupDev> dev;
    int n_up = 0, n_down = 0;
    int nc = 64;                    // column tile of the block GEMM (autotuned)
    std::vector<int> nc_phase;      // per-phase tiles chosen by the tuner (empty: nc everywhere)
    bool use_graph = true;
    // graph cache
    hipGraphExec_t exec = nullptr;
    hipGraph_t graph = nullptr;
    std::string key;
    hipStream_t cap_stream = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    std::string cols_key;           // column configuration the task lists were built for
    std::map<int64_t, std::vector<int>> tile_for_rhs;   // per-phase tiles tuned inside solves, by RHS count
    ~h2_group_s();
};

namespace h2 {

static std::mutex g_groups_mu;
static std::set<h2_group> g_groups;

static size_t a256(size_t b) { return (b + 255) & ~size_t(255); }

// Phases of a group, concatenated over members (absolute device pointers).
static void group_phases(h2_group g) {
    g->n_up = 0;
    g->n_down = 0;
    for (auto& m : g->members) {
        g->n_up = std::max<int>(g->n_up, int(m.B->up.size()));
        g->n_down = std::max<int>(g->n_down, int(m.B->down.size()));
    }
    const int nph = 3 + g->n_up + g->n_down;
    g->host.assign(nph, GPhase());
    // p + off as integer arithmetic: the sizing passes build the same tables before
    // any buffer exists, and offsetting a null pointer is undefined
    auto at = [](auto* p, int64_t off) {
        using T = std::remove_pointer_t<decltype(p)>;
        return reinterpret_cast<T*>(reinterpret_cast<uintptr_t>(p) + uintptr_t(off) * sizeof(T));
    };
    auto rel_phase = [&](int mi, const RelPhase& R, GPhase& G) {
        BatchHost* B = g->members[mi].B;
        const int64_t cols = B->max_cols;
        auto obase = [&](int kind) -> float* { return kind == 0 ? B->Xf : kind == 1 ? B->Yhf : B->Yf; };
        auto orows = [&](int kind) -> int64_t { return kind == 2 ? B->urows : B->crows; };
        auto bbase = [&](int kind) -> uint16_t* { return kind == 0 ? B->Ub : kind == 1 ? B->Xb : B->Yhb; };
        auto brows = [&](int kind) -> int64_t { return kind == 0 ? B->urows : B->crows; };
        const int tbase = int(G.terms.size());
        for (const RelTerm& t : R.terms) {
            BTerm T{};
            T.a = at(B->arena, t.a);
            T.bld = brows(t.b_kind);
            T.bps = T.bld * cols;
            T.b = at(bbase(t.b_kind), t.b_row);
            T.kp = t.kp;
            G.terms.push_back(T);
        }
        for (const RelOwner& o : R.owners) {
            BOwner O{};
            O.ld = orows(o.out_kind);
            O.ps = O.ld * cols;
            O.out = at(obase(o.out_kind), o.out_row);
            O.mp = o.mp;
            O.t0 = tbase + o.t0;
            O.nt = o.nt;
            O.acc = o.acc;
            G.owners.push_back(O);
            G.owner_member.push_back(mi);
        }
        if (R.split_kind >= 0 && R.split_rows > 0) {
            SplitSeg S{};
            const bool x = R.split_kind == 0;
            S.src = x ? B->Xf : B->Yhf;
            S.sld = B->crows;
            S.sps = B->crows * cols;
            S.dst = x ? B->Xb : B->Yhb;
            S.dld = B->crows;
            S.dps = B->crows * cols;
            S.r0 = int(R.split_r0);
            S.nrows = int(R.split_rows);
            G.splits.push_back(S);
        }
    };
    for (int mi = 0; mi < int(g->members.size()); ++mi) {
        BatchHost* B = g->members[mi].B;
        rel_phase(mi, B->leaf, g->host[0]);
        for (int s = 0; s < int(B->up.size()); ++s) rel_phase(mi, B->up[s], g->host[1 + s]);
        rel_phase(mi, B->coup, g->host[1 + g->n_up]);
        for (int s = 0; s < int(B->down.size()); ++s) rel_phase(mi, B->down[s], g->host[2 + g->n_up + s]);
        rel_phase(mi, B->near, g->host[2 + g->n_up + g->n_down]);
    }
}

static size_t group_layout(h2_group g, char* base, bool assign) {
    size_t off = 0;
    auto take = [&](size_t bytes) -> char* {
        char* p = base ? base + off : nullptr;
        off += a256(std::max<size_t>(bytes, 1));
        return p;
    };
    if (assign) g->dev.assign(g->host.size(), GroupDev());
    for (size_t i = 0; i < g->host.size(); ++i) {
        const GPhase& G = g->host[i];
        int max_tasks = 0;
        for (size_t o = 0; o < G.owners.size(); ++o) {
            const int cols = g->members[G.owner_member[o]].B->max_cols;
            max_tasks += (cols + 31) / 32;
        }
        GroupDev D;
        D.owners = (BOwner*)take(G.owners.size() * sizeof(BOwner));
        D.terms = (BTerm*)take(G.terms.size() * sizeof(BTerm));
        D.splits = (SplitSeg*)take(G.splits.size() * sizeof(SplitSeg));
        D.split_cols = (int*)take(G.splits.size() * sizeof(int));
        D.tasks = (int2*)take(size_t(max_tasks) * sizeof(int2));
        D.owner_cols = (int*)take(G.owners.size() * sizeof(int));
        D.n_owners = int(G.owners.size());
        D.n_terms = int(G.terms.size());
        D.n_splits = int(G.splits.size());
        D.max_tasks = max_tasks;
        if (assign) g->dev[i] = D;
    }
    return off + 256;
}

size_t group_bytes(h2_group proto) { return group_layout(proto, nullptr, false); }

static void drop_graph(h2_group g) {
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    g->exec = nullptr;
    g->graph = nullptr;
    g->key.clear();
}

}  // namespace h2

h2_group_s::~h2_group_s() {
    h2::drop_graph(this);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
}

namespace h2 {

// Upload owner/term/split lists (once, at group build).
static hipError_t group_upload(h2_group g, hipStream_t s) {
    for (size_t i = 0; i < g->host.size(); ++i) {
        const GPhase& G = g->host[i];
        GroupDev& D = g->dev[i];
        hipError_t e;
        if (!G.owners.empty() &&
            (e = hipMemcpyAsync(D.owners, G.owners.data(), G.owners.size() * sizeof(BOwner), hipMemcpyHostToDevice, s)) != hipSuccess)
            return e;
        if (!G.terms.empty() &&
            (e = hipMemcpyAsync(D.terms, G.terms.data(), G.terms.size() * sizeof(BTerm), hipMemcpyHostToDevice, s)) != hipSuccess)
            return e;
        if (!G.splits.empty() &&
            (e = hipMemcpyAsync(D.splits, G.splits.data(), G.splits.size() * sizeof(SplitSeg), hipMemcpyHostToDevice, s)) != hipSuccess)
            return e;
    }
    return hipStreamSynchronize(s);
}

static int phase_tile(h2_group g, size_t phase) {
    return phase < g->nc_phase.size() ? g->nc_phase[phase] : g->nc;
}

// Task lists (owner, first column) for the current column counts.
static hipError_t group_tasks(h2_group g, hipStream_t s) {
    std::string key = std::to_string(g->nc);
    for (int t : g->nc_phase) key += "/" + std::to_string(t);
    for (auto& m : g->members) key += "," + std::to_string(m.ncols);
    if (key == g->cols_key) return hipSuccess;
    for (size_t i = 0; i < g->host.size(); ++i) {
        const GPhase& G = g->host[i];
        GroupDev& D = g->dev[i];
        std::vector<int2> tasks;
        std::vector<int> ocols(G.owners.size());
        for (size_t o = 0; o < G.owners.size(); ++o) {
            const int cols = g->members[G.owner_member[o]].ncols;
            ocols[o] = cols;
            for (int c0 = 0; c0 < cols; c0 += phase_tile(g, i)) tasks.push_back(make_int2(int(o), c0));
        }
        std::vector<int> scols;
        int64_t mx = 0;
        for (const SplitSeg& S : G.splits) {      // columns of the member whose planes a segment reads
            int cols = 0;
            for (auto& m : g->members)
                if (S.src == m.B->Xf || S.src == m.B->Yhf) cols = m.ncols;
            scols.push_back(cols);
            mx = std::max<int64_t>(mx, int64_t(S.nrows) * cols);
        }
        if (int(tasks.size()) > D.max_tasks) return hipErrorInvalidValue;
        D.n_tasks = int(tasks.size());
        D.max_split_elems = mx;
        hipError_t e;
        if (!tasks.empty() &&
            (e = hipMemcpyAsync(D.tasks, tasks.data(), tasks.size() * sizeof(int2), hipMemcpyHostToDevice, s)) != hipSuccess)
            return e;
        if (!ocols.empty() &&
            (e = hipMemcpyAsync(D.owner_cols, ocols.data(), ocols.size() * sizeof(int), hipMemcpyHostToDevice, s)) != hipSuccess)
            return e;
        if (!scols.empty() &&
            (e = hipMemcpyAsync(D.split_cols, scols.data(), scols.size() * sizeof(int), hipMemcpyHostToDevice, s)) != hipSuccess)
            return e;
    }
    hipError_t e = hipStreamSynchronize(s);
    if (e == hipSuccess) g->cols_key = key;
    return e;
}

// The whole batched product of every member, phase by phase.  ev (optional, two
// events per phase) brackets each phase's block GEMM for the tuner.
static hipError_t group_launch(h2_group g, int op, const void* const* x, void* const* y, const int64_t* ld,
                               hipStream_t s, const std::vector<hipEvent_t>* ev = nullptr) {
    hipError_t e;
    for (size_t mi = 0; mi < g->members.size(); ++mi) {
        const GroupMember& m = g->members[mi];
        if (m.ncols == 0) continue;
        const DevH2& D = m.h->dev;
        if ((e = launch_prologue_b(D.n_vox, D.perm, m.B->prow_dev, D.chi, (const float2*)x[mi], ld[mi], m.ncols,
                                   m.B->Ub, m.B->urows, m.B->urows * m.B->max_cols, op, s)) != hipSuccess)
            return e;
    }
    for (size_t i = 0; i < g->host.size(); ++i) {
        GroupDev& P = g->dev[i];
        if (ev && (e = hipEventRecord((*ev)[2 * i], s)) != hipSuccess) return e;
        if ((e = launch_bgemm(phase_tile(g, i), P.owners, P.terms, P.tasks, P.n_tasks, P.owner_cols, s)) != hipSuccess)
            return e;
        if (ev && (e = hipEventRecord((*ev)[2 * i + 1], s)) != hipSuccess) return e;
        if ((e = launch_split(P.splits, P.n_splits, int(std::min<int64_t>(P.max_split_elems, 1 << 30)),
                              P.split_cols, s)) != hipSuccess)
            return e;
    }
    for (size_t mi = 0; mi < g->members.size(); ++mi) {
        const GroupMember& m = g->members[mi];
        if (m.ncols == 0) continue;
        const DevH2& D = m.h->dev;
        const float alpha = float(D.sigma * D.k * D.k * D.volume);
        if ((e = launch_epilogue_b(D.n_vox, D.perm, m.B->prow_dev, m.B->Yf, m.B->urows, m.B->urows * m.B->max_cols,
                                   (const float2*)x[mi], ld[mi], (float2*)y[mi], ld[mi], m.ncols, op, alpha, s)) !=
            hipSuccess)
            return e;
    }
    return hipSuccess;
}

h2_status group_run(h2_group g, int op, const void* const* x, void* const* y, const int64_t* n_rhs, const int64_t* ld,
                    hipStream_t s) {
    for (size_t mi = 0; mi < g->members.size(); ++mi) {
        GroupMember& m = g->members[mi];
        const int64_t N = int64_t(m.h->dev.n_vox) * kNcomp;
        if (n_rhs[mi] < 0 || 3 * n_rhs[mi] > m.B->max_cols) return handle_fail(H2_ERR_INVALID_ARG, "n_rhs out of range for a member");
        if (n_rhs[mi] > 0 && (!x[mi] || !y[mi] || ld[mi] < N)) return handle_fail(H2_ERR_INVALID_ARG, "bad vector of a member");
        if (n_rhs[mi] > 0 && ((reinterpret_cast<uintptr_t>(x[mi]) | reinterpret_cast<uintptr_t>(y[mi])) % 8))
            return handle_fail(H2_ERR_INVALID_ARG, "misaligned vector");
        m.ncols = int(3 * n_rhs[mi]);
    }
    hipError_t e = group_tasks(g, s);
    if (e != hipSuccess) return handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
    if (!g->use_graph) {
        e = group_launch(g, op, x, y, ld, s);
        if (e != hipSuccess) return handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
        return H2_OK;
    }
    // graph keyed by pointers, columns and op; launched on a private stream ordered after s
    std::string key = g->cols_key + "|" + std::to_string(op);
    for (size_t mi = 0; mi < g->members.size(); ++mi)
        key += "|" + std::to_string(reinterpret_cast<uintptr_t>(x[mi])) + "," +
               std::to_string(reinterpret_cast<uintptr_t>(y[mi])) + "," + std::to_string(ld[mi]);
    if (!g->cap_stream) {
        if ((e = hipStreamCreateWithFlags(&g->cap_stream, hipStreamNonBlocking)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&g->ev_in, hipEventDisableTiming)) != hipSuccess ||
            (e = hipEventCreateWithFlags(&g->ev_out, hipEventDisableTiming)) != hipSuccess)
            return handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
    }
    if (key != g->key) {
        drop_graph(g);
        if ((e = hipStreamBeginCapture(g->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
            return handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
        hipError_t le = group_launch(g, op, x, y, ld, g->cap_stream);
        hipGraph_t graph = nullptr;
        e = hipStreamEndCapture(g->cap_stream, &graph);
        if (le != hipSuccess || e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return handle_fail(H2_ERR_DEVICE, hipGetErrorString(le != hipSuccess ? le : e));
        }
        if ((e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0)) != hipSuccess) {
            (void)hipGraphDestroy(graph);
            return handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
        }
        g->graph = graph;
        g->key = key;
    }
    if ((e = hipEventRecord(g->ev_in, s)) != hipSuccess || (e = hipStreamWaitEvent(g->cap_stream, g->ev_in, 0)) != hipSuccess ||
        (e = hipGraphLaunch(g->exec, g->cap_stream)) != hipSuccess || (e = hipEventRecord(g->ev_out, g->cap_stream)) != hipSuccess ||
        (e = hipStreamWaitEvent(s, g->ev_out, 0)) != hipSuccess)
        return handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
    return H2_OK;
}

h2_status group_create(const h2_handle* hs, int n, void* mem, size_t bytes, hipStream_t s, h2_group* out) {
    h2_group g = new h2_group_s();
    for (int i = 0; i < n; ++i) g->members.push_back({hs[i], hs[i]->batch, 0});
    group_phases(g);
    const size_t need = group_layout(g, nullptr, false);
    char* base = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(mem) + 255) & ~uintptr_t(255));
    if (bytes < need + size_t(base - reinterpret_cast<char*>(mem))) {
        delete g;
        return handle_fail(H2_ERR_OOM, "group buffer too small");
    }
    group_layout(g, base, true);
    hipError_t e = group_upload(g, s);
    if (e != hipSuccess) {
        delete g;
        return handle_fail(H2_ERR_DEVICE, hipGetErrorString(e));
    }
    {
        std::lock_guard<std::mutex> lk(g_groups_mu);
        g_groups.insert(g);
    }
    *out = g;
    return H2_OK;
}

size_t group_need_batch(BatchHost* B) {
    h2_group_s tmp;
    tmp.members.push_back({nullptr, B, 0});
    group_phases(&tmp);
    return group_layout(&tmp, nullptr, false);
}

size_t group_need(const h2_handle* hs, int n) {
    h2_group_s tmp;
    for (int i = 0; i < n; ++i) tmp.members.push_back({hs[i], hs[i]->batch, 0});
    group_phases(&tmp);
    return group_layout(&tmp, nullptr, false);
}

static bool group_ok(h2_group g) {
    if (!g) return false;
    std::lock_guard<std::mutex> lk(g_groups_mu);
    return g_groups.count(g) && g->magic == 0x48324752u;
}

void group_destroy(h2_group g) {
    if (!group_ok(g)) return;
    {
        std::lock_guard<std::mutex> lk(g_groups_mu);
        g_groups.erase(g);
    }
    g->magic = 0;
    delete g;
}

}  // namespace h2

using namespace h2;

extern "C" {

h2_status h2_group_plan(const h2_handle* members, int32_t n, size_t* dev_bytes) {
    if (!members || n < 1 || !dev_bytes) return handle_fail(H2_ERR_INVALID_ARG, "null or empty member list");
    for (int i = 0; i < n; ++i) {
        if (!handle_live(members[i])) return handle_fail(H2_ERR_BAD_HANDLE, "invalid member handle");
        if (!members[i]->batch) return handle_fail(H2_ERR_INVALID_ARG, "member built without the BF16X3 tier");
    }
    *dev_bytes = group_need(members, n) + 256;
    return H2_OK;
}

h2_status h2_group_build(const h2_handle* members, int32_t n, void* dev_buffer, size_t dev_bytes, void* stream,
                         h2_group* out) {
    if (!out) return handle_fail(H2_ERR_INVALID_ARG, "null output");
    *out = nullptr;
    size_t need = 0;
    h2_status st = h2_group_plan(members, n, &need);
    if (st != H2_OK) return st;
    if (!dev_buffer) return handle_fail(H2_ERR_INVALID_ARG, "null device buffer");
    return group_create(members, n, dev_buffer, dev_bytes, reinterpret_cast<hipStream_t>(stream), out);
}

h2_status h2_group_matvec(h2_group g, h2_op op, const void* const* x, void* const* y, const int64_t* n_rhs,
                          const int64_t* ld, void* stream) {
    if (!group_ok(g)) return handle_fail(H2_ERR_BAD_HANDLE, "invalid group");
    if (op != H2_OP_G && op != H2_OP_Z) return handle_fail(H2_ERR_INVALID_ARG, "unknown op");
    if (!x || !y || !n_rhs || !ld) return handle_fail(H2_ERR_INVALID_ARG, "null argument");
    for (auto& m : g->members)
        if (!handle_live(m.h)) return handle_fail(H2_ERR_BAD_HANDLE, "a member handle was destroyed");
    return group_run(g, int(op), x, y, n_rhs, ld, reinterpret_cast<hipStream_t>(stream));
}

h2_status h2_group_tune(h2_group g, h2_op op, const void* const* x, void* const* y, const int64_t* n_rhs,
                        const int64_t* ld, void* stream, int32_t* tile) {
    if (!group_ok(g)) return handle_fail(H2_ERR_BAD_HANDLE, "invalid group");
    if (!tile) return handle_fail(H2_ERR_INVALID_ARG, "null tile output");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const int cand[3] = {32, 64, 128};
    const size_t np = g->host.size();
    std::vector<hipEvent_t> ev(2 * np, nullptr);
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            for (auto& f : ev)
                if (f) (void)hipEventDestroy(f);
            return handle_fail(H2_ERR_DEVICE, "event creation failed");
        }
    auto release = [&]() {
        for (auto& f : ev) (void)hipEventDestroy(f);
    };
    // every phase's block GEMM timed at every tile width (three products each); each phase keeps its fastest
    std::vector<double> best(np, 1e300);
    std::vector<int> pick(np, g->nc);
    const bool graph = g->use_graph;
    g->use_graph = false;
    for (int c : cand) {
        g->nc = c;
        g->nc_phase.clear();
        h2_status st = group_run(g, int(op), x, y, n_rhs, ld, s);   // warm-up (also builds the task lists)
        if (st != H2_OK) { g->use_graph = graph; release(); return st; }
        std::vector<double> t(np, 0.0);
        for (int r = 0; r < 3; ++r) {
            hipError_t e = group_launch(g, int(op), x, y, ld, s, &ev);
            if (e == hipSuccess) e = hipStreamSynchronize(s);
            if (e != hipSuccess) { g->use_graph = graph; release(); return handle_fail(H2_ERR_DEVICE, "tuning run failed"); }
            for (size_t i = 0; i < np; ++i) {
                float ms = 0.f;
                if (hipEventElapsedTime(&ms, ev[2 * i], ev[2 * i + 1]) == hipSuccess) t[i] += ms;
            }
        }
        for (size_t i = 0; i < np; ++i)
            if (t[i] < best[i]) { best[i] = t[i]; pick[i] = c; }
    }
    release();
    g->use_graph = graph;
    g->nc = np ? pick[np - 1] : 64;      // the near-field phase's tile, reported
    g->nc_phase = pick;
    drop_graph(g);
    g->cols_key.clear();
    *tile = g->nc;
    return H2_OK;
}

h2_status h2_group_set(h2_group g, int32_t tile, int32_t use_graph) {
    if (!group_ok(g)) return handle_fail(H2_ERR_BAD_HANDLE, "invalid group");
    if (tile != 0 && tile != 32 && tile != 64 && tile != 128) return handle_fail(H2_ERR_INVALID_ARG, "tile must be 32, 64 or 128");
    if (tile) {
        g->nc = tile;
        g->nc_phase.clear();
    }
    g->use_graph = use_graph != 0;
    drop_graph(g);
    g->cols_key.clear();
    return H2_OK;
}

void h2_group_destroy(h2_group g) { group_destroy(g); }

}  // extern "C"

namespace h2 {

// Tile for a single-member group at n_rhs right-hand sides: tuned on first use
// (timing the three tiles on the given buffers, whose values do not matter),
// then reused.  Used by the solvers before their first product.
h2_status group_autotile(h2_group g, const void* x, void* y, int64_t n_rhs, int64_t ld, hipStream_t s) {
    if (!group_ok(g)) return handle_fail(H2_ERR_BAD_HANDLE, "invalid group");
    auto it = g->tile_for_rhs.find(n_rhs);
    if (it != g->tile_for_rhs.end()) {
        if (g->nc_phase != it->second) {
            g->nc_phase = it->second;
            drop_graph(g);
            g->cols_key.clear();
        }
        return H2_OK;
    }
    const void* xs[1] = {x};
    void* ys[1] = {y};
    const int64_t nr[1] = {n_rhs}, lds[1] = {ld};
    int32_t tile = 0;
    h2_status st = h2_group_tune(g, H2_OP_Z, xs, ys, nr, lds, s, &tile);
    if (st != H2_OK) return st;
    g->tile_for_rhs[n_rhs] = g->nc_phase;
    return H2_OK;
}

}  // namespace h2
