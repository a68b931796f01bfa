// batch.hip -- batched cavities: task packing, persistent-kernel launches,
// HIP-graph replay of k round trips, autotuning with a JSON cache.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <set>
#include <string>
#include <vector>

#include "batch.hpp"
#include "host.hpp"

namespace lsr {

GroupInfo group_256();
GroupInfo group_384();
GroupInfo group_512();
GroupInfo group_768();
GroupInfo group_1024();
GroupInfo group_2048();
GroupInfo group_4096();
GroupInfo group_small();
GroupInfo group_512r();
GroupInfo group_1024r();
GroupInfo group_1024t();
GroupInfo group_2048r();
GroupInfo group_4096w();
GroupInfo group_256l();
GroupInfo group_any_256();
GroupInfo group_any_384();
GroupInfo group_any_512();
GroupInfo group_any_768();
GroupInfo group_any_1024();
GroupInfo group_any_2048();
GroupInfo group_any_4096();
GroupInfo group_anyr_256();
GroupInfo group_anyr_384();
GroupInfo group_anyr_512();
GroupInfo group_anyr_768();
GroupInfo group_anyr_1024();
GroupInfo group_anyr_2048();
GroupInfo group_anyr_4096();
GroupInfo group_fix1_256();
GroupInfo group_fix2_256();
GroupInfo group_fix1_384();
GroupInfo group_fix2_384();
GroupInfo group_fix1_512();
GroupInfo group_fix2_512();
GroupInfo group_fix1_768();
GroupInfo group_fix2_768();
GroupInfo group_fix1_1024();
GroupInfo group_fix2_1024();
GroupInfo group_fix1_2048();
GroupInfo group_fix2_2048();
GroupInfo group_fix1_4096();
GroupInfo group_fix2_4096();

static const std::vector<GroupInfo>& groups() {
    static const std::vector<GroupInfo> g = {group_256(),  group_384(),  group_512(),
                                             group_768(),  group_1024(), group_2048(),
                                             group_4096(), group_small(), group_512r(),
                                             group_1024r(), group_1024t(), group_2048r(), group_4096w(), group_256l(),
                                             group_any_256(), group_any_384(), group_any_512(),
                                             group_any_768(), group_any_1024(), group_any_2048(),
                                             group_any_4096(), group_anyr_256(), group_anyr_384(),
                                             group_anyr_512(), group_anyr_768(), group_anyr_1024(),
                                             group_anyr_2048(), group_anyr_4096(),
                                             group_fix1_256(), group_fix2_256(), group_fix1_384(), group_fix2_384(), group_fix1_512(), group_fix2_512(), group_fix1_768(), group_fix2_768(), group_fix1_1024(), group_fix2_1024(), group_fix1_2048(), group_fix2_2048(), group_fix1_4096(), group_fix2_4096()};
    return g;
}
int group_count() { return (int)groups().size(); }
const GroupInfo* group_at(int i) { return (i >= 0 && i < group_count()) ? &groups()[i] : nullptr; }

int row_blocks(int N) {
    ShapeInfo s;
    if (!shape_for(N, false, &s)) return 0;
    return N / s.LPW;
}

// Task order of one trip for cavities with the given row-block counts: all
// row tasks in cavity order; the column tasks of cavity c follow once `lag`
// further row tasks have been emitted after c's last row task (or at the
// end).  Every column task therefore has a larger ticket than each row task
// it depends on.
static void pack(const std::vector<int>& nrb, int lag, bool with_cols, std::vector<int4>& out) {
    out.clear();
    const int n = (int)nrb.size();
    std::vector<long> end(n);
    long total = 0;
    for (int c = 0; c < n; ++c) {
        total += nrb[c];
        end[c] = total;
    }
    int next_col = 0;
    long emitted_rows = 0;
    auto flush_cols = [&](bool all) {
        while (with_cols && next_col < n && (all || end[next_col] + lag <= emitted_rows)) {
            for (int b = 0; b < nrb[next_col]; ++b) out.push_back(int4{next_col, TASK_COL, b, 0});
            ++next_col;
        }
    };
    for (int c = 0; c < n; ++c)
        for (int b = 0; b < nrb[c]; ++b) {
            out.push_back(int4{c, TASK_ROW, b, 0});
            ++emitted_rows;
            flush_cols(false);
        }
    flush_cols(true);
}

static int default_lag() { return 2048; }

struct Tune {
    int engine = 1;       // 0 persistent kernel per trip, 1 grouped launch per pass,
                          // 2 grouped and software-pipelined (single-size groups)
    int variant = 0;      // kernel variant (register budget) of each group
    int wgs_per_cu = 0;   // 0 = occupancy limit
    int chunk = 2;
    int lag = -1;         // -1 = default
    int graph_k = 16;     // trips per captured graph; 0 = eager
    int merge = 0;        // 0 one group (kernel) per grid size; 1 one group per
                          // workgroup size, uneven sizes sharing one kernel
    int shape = 0;        // FFT plan of single-size groups: 0 the size's default,
                          // k > 0 its alternative plan k where one is compiled
};

// --------------------------------------------------------------- cache ----
// {"<key>": {"wgs_per_cu": a, "chunk": b, "lag": c, "graph_k": d}, ...}
static std::string cache_path(const char* p) {
    if (p && *p) return p;
    const char* e = getenv("LSR_TUNE_CACHE");
    return e ? e : "";
}

static std::map<std::string, Tune> cache_read(const std::string& path) {
    std::map<std::string, Tune> m;
    if (path.empty()) return m;
    FILE* f = fopen(path.c_str(), "rb");
    if (!f) return m;
    std::string s;
    char buf[4096];
    size_t k;
    while ((k = fread(buf, 1, sizeof buf, f)) > 0) s.append(buf, k);
    fclose(f);
    size_t i = 0;
    while ((i = s.find('"', i)) != std::string::npos) {
        const size_t j = s.find('"', i + 1);
        if (j == std::string::npos) break;
        const std::string key = s.substr(i + 1, j - i - 1);
        const size_t ob = s.find('{', j), cb = s.find('}', j);
        if (ob == std::string::npos || cb == std::string::npos || ob > cb) { i = j + 1; continue; }
        const std::string body = s.substr(ob + 1, cb - ob - 1);
        Tune t;
        auto get = [&](const char* name, int& v) {
            const std::string q = std::string("\"") + name + "\"";
            const size_t p = body.find(q);
            if (p != std::string::npos) {
                const size_t c = body.find(':', p);
                if (c != std::string::npos) v = atoi(body.c_str() + c + 1);
            }
        };
        get("engine", t.engine);
        get("variant", t.variant);
        get("wgs_per_cu", t.wgs_per_cu);
        get("chunk", t.chunk);
        get("lag", t.lag);
        get("graph_k", t.graph_k);
        get("merge", t.merge);
        get("shape", t.shape);
        m[key] = t;
        i = cb + 1;
    }
    return m;
}

static bool cache_write(const std::string& path, const std::map<std::string, Tune>& m) {
    if (path.empty()) return true;
    const std::string tmp = path + ".tmp";
    FILE* f = fopen(tmp.c_str(), "wb");
    if (!f) return false;
    fprintf(f, "{\n");
    size_t n = 0;
    for (const auto& kv : m) {
        fprintf(f,
                "  \"%s\": {\"engine\": %d, \"variant\": %d, \"wgs_per_cu\": %d, \"chunk\": %d, \"lag\": %d, "
                "\"graph_k\": %d, \"merge\": %d, \"shape\": %d}%s\n",
                kv.first.c_str(), kv.second.engine, kv.second.variant, kv.second.wgs_per_cu, kv.second.chunk,
                kv.second.lag, kv.second.graph_k, kv.second.merge, kv.second.shape, ++n < m.size() ? "," : "");
    }
    fprintf(f, "}\n");
    fclose(f);
    return rename(tmp.c_str(), path.c_str()) == 0;
}

}  // namespace lsr

using namespace lsr;

struct BatchGroup {
    const GroupInfo* g = nullptr;
    std::vector<int> cav;            // batch indices of this group's cavities
    CavDesc* d_desc = nullptr;       // per cavity of the group
    int4* d_tasks = nullptr;         // trip tasks (rows + columns)
    int ntasks = 0;
    int4* d_last = nullptr;          // row tasks only (last trip; grouped row pass)
    int nlast = 0;
    int4* d_cols = nullptr;          // column tasks only (grouped column pass)
    int ncols = 0;
    int sheets = 1;                  // gain sheets per round trip of the group's cavities
    unsigned* d_ctrl = nullptr;
    void* d_tw[8] = {};              // twiddles of each size of the group, for its FFT plan
    int occ[4] = {1, 1, 1, 1};   // resident workgroups per CU of each variant
    int occ_pipe[4][2] = {};     // same for the pipelined row / column pass
};

struct lsr_batch_s {
    int device = 0;
    int cus = 256;
    hipStream_t user = nullptr;      // stream of plans[0]
    hipStream_t stream = nullptr;    // private stream (graph capture needs a non-null stream)
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    std::vector<lsr_plan> plans;
    std::vector<BatchGroup> grp;
    std::vector<void*> lastE, lastN;
    std::vector<unsigned> lastVer;   // plan descriptor versions of the last upload
    std::vector<int> models;         // the plans' group codes (model, roughness, transfer
                                     // function) when grouped
    Tune tune;
    std::string key;
    // captured launch sequences, reused across calls (see run_trips)
    struct Graph {
        int kind = 0;                    // GRAPH_MID or GRAPH_CALL
        int len = 0;                     // trips
        hipGraphExec_t exec = nullptr;
        unsigned long long used = 0;     // last use (for eviction)
    };
    std::vector<Graph> graphs;
    unsigned long long graph_clock = 0;
    bool launched = false;               // a graph may still be in flight on stream
};

static void groups_free(lsr_batch_s* b) {
    for (auto& g : b->grp) {
        if (g.d_desc) (void)hipFree(g.d_desc);
        if (g.d_tasks) (void)hipFree(g.d_tasks);
        if (g.d_last) (void)hipFree(g.d_last);
        if (g.d_cols) (void)hipFree(g.d_cols);
        if (g.d_ctrl) (void)hipFree(g.d_ctrl);
        for (void* t : g.d_tw)
            if (t) (void)hipFree(t);
    }
    b->grp.clear();
    b->lastE.clear();
    b->lastN.clear();
}

static void drop_graphs(lsr_batch_s* b);

static void batch_free(lsr_batch_s* b) {
    drop_graphs(b);
    groups_free(b);
    if (b->ev_in) (void)hipEventDestroy(b->ev_in);
    if (b->ev_out) (void)hipEventDestroy(b->ev_out);
    if (b->stream) (void)hipStreamDestroy(b->stream);
}

static std::string batch_key(const std::vector<lsr_plan>& plans) {
    std::map<int, int> cnt;
    for (auto* p : plans) cnt[p->N]++;
    std::string k = "gfx950:batch:";
    for (auto& kv : cnt) k += std::to_string(kv.first) + "x" + std::to_string(kv.second) + ";";
    return k;
}

// Row (= column) blocks of a size-N cavity under its group's FFT plan.
static int group_blocks(const BatchGroup& g, int N) {
    for (int k = 0; k < g.g->nsizes; ++k)
        if (g.g->sizes[k] == N) return N / g.g->shapes[k].LPW;
    return 0;
}

// What a plan's group must match: its local-step code (model, roughness),
// whether it has a general transfer function, and its number of gain sheets.
static int group_code(const lsr_plan_s* q) { return q->d.model | (q->d_trans ? 1 << 8 : 0) | (q->slices << 9); }

// After a failed regroup or repack: no group is left half built.  The
// recorded local-step codes are cleared too, so the next call regroups
// (regroup_if_models_changed) or reports the failure again.
static int groups_invalidate(lsr_batch_s* b, int rc) {
    groups_free(b);
    b->models.clear();
    return rc;
}

// (Re)build the task lists of every group for the current tuning.
static int batch_pack_groups(lsr_batch_s* b) {
    const int lag = b->tune.lag >= 0 ? b->tune.lag : default_lag();
    for (auto& g : b->grp) {
        std::vector<int> nrb;
        for (int c : g.cav) nrb.push_back(group_blocks(g, b->plans[c]->N));
        std::vector<int4> t, l, cols;
        pack(nrb, lag, true, t);
        pack(nrb, 0, false, l);
        for (const int4& x : t)
            if (x.y == TASK_COL) cols.push_back(x);
        if (g.d_tasks) (void)hipFree(g.d_tasks);
        if (g.d_last) (void)hipFree(g.d_last);
        if (g.d_cols) (void)hipFree(g.d_cols);
        g.d_tasks = g.d_last = g.d_cols = nullptr;
        g.ntasks = g.nlast = g.ncols = 0;
        if (dev_malloc((void**)&g.d_tasks, t.size() * sizeof(int4)) != hipSuccess ||
            dev_malloc((void**)&g.d_last, l.size() * sizeof(int4)) != hipSuccess ||
            dev_malloc((void**)&g.d_cols, cols.size() * sizeof(int4)) != hipSuccess)
            return set_err(LSR_ENOMEM, "task table allocation failed");
        LSR_HIP(hipMemcpy(g.d_tasks, t.data(), t.size() * sizeof(int4), hipMemcpyHostToDevice));
        LSR_HIP(hipMemcpy(g.d_last, l.data(), l.size() * sizeof(int4), hipMemcpyHostToDevice));
        LSR_HIP(hipMemcpy(g.d_cols, cols.data(), cols.size() * sizeof(int4), hipMemcpyHostToDevice));
        g.ntasks = (int)t.size();
        g.nlast = (int)l.size();
        g.ncols = (int)cols.size();
    }
    return LSR_OK;
}

static int batch_pack(lsr_batch_s* b) {
    const int rc = batch_pack_groups(b);
    return rc == LSR_OK ? rc : groups_invalidate(b, rc);
}

// Cavities -> groups.  merge = 0: one group per grid size (each kernel
// specialised for its size: registers and LDS of that size only), with the
// size's alternative FFT plan tune.shape where one is compiled; merge = 1:
// one group per workgroup size, the smallest compiled kernel of default plans
// that covers all the part's sizes (uneven sizes advance in one launch).
// Allocates the groups' descriptor and control blocks (and the twiddles of an
// alternative plan) and packs their task lists.
static int batch_partition_groups(lsr_batch_s* b) {
    groups_free(b);
    // sizes with a cavity of another local-step code than the default, or
    // with a general transfer function, run on kernels for that size alone
    // (key -(64N + level)): level ANY_FIXED + m when every cavity of the size
    // has model m, a smooth mirror and the propagator or filter, else 1
    // (kernels that read each cavity's model and propagator kind) or 2 when
    // one has a rough mirror (model and roughness read per cavity)
    b->models.clear();
    std::map<int, int> level;
    std::map<int, std::set<int>> codes;
    std::set<int> with_trans;
    for (auto* q : b->plans) {
        b->models.push_back(group_code(q));
        int l = (q->d.model & MODEL_ROUGH) ? 2 : q->d.model != 0 ? 1 : 0;
        if (q->d_trans) {
            l = std::max(l, 1);
            with_trans.insert(q->N);
        }
        level[q->N] = std::max(level[q->N], l);
        codes[q->N].insert(q->d.model);
    }
    for (auto& kv : level)
        if (kv.second == 1 && codes[kv.first].size() == 1 && !with_trans.count(kv.first))
            kv.second = ANY_FIXED + *codes[kv.first].begin();
    // one group per number of gain sheets too: a group's sheet steps are its
    // launches, sheet-major descriptors of its cavities
    std::map<std::pair<int, int>, std::vector<int>> parts;
    for (int i = 0; i < (int)b->plans.size(); ++i) {
        ShapeInfo s;
        shape_for(b->plans[i]->N, false, &s);
        const int N = b->plans[i]->N;
        parts[{b->plans[i]->slices, level[N] ? -(64 * N + level[N]) : b->tune.merge ? s.threads : N}].push_back(i);
    }
    for (auto& kv : parts) {
        const GroupInfo* best = nullptr;
        const int sheets = kv.first.first, pkey = kv.first.second;
        const bool any = pkey < 0;
        const int any_level = any ? (-pkey) % 64 : 0;
        const bool merged = b->tune.merge && !any;
        const int key = any ? (-pkey) / 64 : pkey;
        const int want = (merged || any) ? 0 : b->tune.shape;
        for (int pass = 0; pass < 2 && !best; ++pass)
        for (int gi = 0; gi < group_count() && !best; ++gi) {
            const GroupInfo* g = group_at(gi);
            if (g->any_model != any_level) continue;
            if (merged ? g->threads != key : (g->nsizes != 1 || g->sizes[0] != key)) continue;
            // the wanted plan first, else the default one
            if (g->alt != (pass == 0 ? want : 0)) continue;
            bool all = true;
            for (int c : kv.second) {
                bool in = false;
                for (int k = 0; k < g->nsizes; ++k) in |= g->sizes[k] == b->plans[c]->N;
                all &= in;
            }
            if (all) best = g;
        }
        if (!best) return set_err(LSR_EUNSUPPORTED, "no compiled group covers this mix of sizes");
        BatchGroup bg;
        bg.g = best;
        bg.cav = kv.second;
        bg.sheets = sheets;
        for (int v = 0; v < best->nvariants; ++v) {
            bg.occ[v] = best->var[v].occupancy();
            if (best->var[v].occupancy_pipe) {
                bg.occ_pipe[v][TASK_ROW] = best->var[v].occupancy_pipe(TASK_ROW);
                bg.occ_pipe[v][TASK_COL] = best->var[v].occupancy_pipe(TASK_COL);
            }
        }
        const size_t ncav = bg.cav.size();
        b->grp.push_back(bg);
        BatchGroup& g = b->grp.back();
        if (dev_malloc((void**)&g.d_desc, (size_t)g.sheets * ncav * sizeof(CavDesc)) != hipSuccess ||
            dev_malloc((void**)&g.d_ctrl, (CTRL_ROWDONE + ncav) * sizeof(unsigned)) != hipSuccess)
            return set_err(LSR_ENOMEM, "batch allocation failed");
        // the twiddles of each size under the group's FFT plan, FP64-built
        // like a plan's own (a plan's table may be of another shape)
        for (int k = 0; k < best->nsizes; ++k) {
            const std::vector<double> tw = build_twiddles(best->shapes[k], false, true);
            std::vector<float> twf(tw.begin(), tw.end());
            if (dev_malloc(&g.d_tw[k], twf.size() * sizeof(float)) != hipSuccess)
                return set_err(LSR_ENOMEM, "batch allocation failed");
            LSR_HIP(hipMemcpy(g.d_tw[k], twf.data(), twf.size() * sizeof(float), hipMemcpyHostToDevice));
        }
        std::vector<unsigned> ctrl(CTRL_ROWDONE + ncav, 0u);
        ctrl[CTRL_NCAV] = (unsigned)ncav;
        if (hipMemcpy(g.d_ctrl, ctrl.data(), ctrl.size() * sizeof(unsigned), hipMemcpyHostToDevice) != hipSuccess)
            return set_err(LSR_EDEVICE, "control block upload failed");
    }
    return batch_pack(b);
}

static int batch_partition(lsr_batch_s* b) {
    const int rc = batch_partition_groups(b);
    return rc == LSR_OK ? rc : groups_invalidate(b, rc);
}

static int variant_of(const lsr_batch_s* b, const BatchGroup& g) {
    const int v = b->tune.variant;
    return (v >= 0 && v < g.g->nvariants) ? v : 0;
}

static int grid_of(const lsr_batch_s* b, const BatchGroup& g) {
    int per_cu = g.occ[variant_of(b, g)];
    if (b->tune.wgs_per_cu > 0 && b->tune.wgs_per_cu < per_cu) per_cu = b->tune.wgs_per_cu;
    return per_cu * b->cus;
}

// One grouped pass (kind TASK_ROW or TASK_COL) of every group.
// Descriptors of gain sheet k of group g (the group's cavities, sheet-major).
static const CavDesc* sheet_descs(const BatchGroup& g, int k) { return g.d_desc + (size_t)k * g.cav.size(); }

static int launch_grouped_pass(lsr_batch_s* b, int mode, int kind, LaunchEvents ev = {}, int sheet = 0) {
    // the groups whose trip has a sheet step `sheet`
    std::vector<size_t> run;
    for (size_t i = 0; i < b->grp.size(); ++i)
        if (sheet < b->grp[i].sheets) run.push_back(i);
    for (size_t j = 0; j < run.size(); ++j) {
        auto& g = b->grp[run[j]];
        const CavDesc* descs = sheet_descs(g, sheet);
        const int v = variant_of(b, g);
        const KernelVariant& kv = g.g->var[v];
        const int4* tasks = kind == TASK_ROW ? g.d_last : g.d_cols;
        const int nt = kind == TASK_ROW ? g.nlast : g.ncols;
        // timestamps: start of the first group's dispatch, end of the last's
        LaunchEvents e;
        if (j == 0) e.start = ev.start;
        if (j + 1 == run.size()) e.stop = ev.stop;
        int rc;
        if (b->tune.engine == 2 && kv.launch_pipe)
            rc = kv.launch_pipe(mode, kind, b->stream, descs, tasks, nt, g.occ_pipe[v][kind] * b->cus, e);
        else
            rc = kv.launch_pass(mode, kind, b->stream, descs, tasks, nt, e);
        if (rc)
            return set_err(LSR_EDEVICE, "%s-pass launch failed: %s", kind == TASK_ROW ? "row" : "column",
                           hipGetErrorString(hipGetLastError()));
    }
    return LSR_OK;
}

// One round trip of every cavity (mode ROW_FIRST or ROW_MID), or the last
// row pass of a call (ROW_LAST).  With m gain sheets a trip is m steps: the
// row pass of sheet k (sheet 0 in `mode`, the others as middle passes), then
// its column pass; the column pass of sheet 0 folds the trip's sums.  Step k
// launches the groups whose cavities have more than k sheets.
static int max_sheets(const lsr_batch_s* b) {
    int m = 1;
    for (const auto& g : b->grp) m = std::max(m, g.sheets);
    return m;
}

static int launch_trip(lsr_batch_s* b, int mode, LaunchEvents ev) {
    const int m = mode == ROW_LAST ? 1 : max_sheets(b);
    int rc = LSR_OK;
    for (int k = 0; k < m && rc == LSR_OK; ++k) {
        const int md = k == 0 ? mode : ROW_MID;
        if (b->tune.engine >= 1) {
            // grouped: every cavity's row blocks, then every cavity's column blocks
            rc = launch_grouped_pass(b, md, TASK_ROW, {}, k);
            if (rc == LSR_OK && md != ROW_LAST) rc = launch_grouped_pass(b, md, TASK_COL, {}, k);
            continue;
        }
        const size_t ng = b->grp.size();
        // the last group with a sheet step k (at k = m - 1 one with m sheets)
        size_t last_g = 0;
        for (size_t i = 0; i < ng; ++i)
            if (k < b->grp[i].sheets) last_g = i;
        for (size_t i = 0; i < ng && rc == LSR_OK; ++i) {
            auto& g = b->grp[i];
            if (k >= g.sheets) continue;
            const bool last = md == ROW_LAST;
            const int nt = last ? g.nlast : g.ntasks;
            const int grid = std::min(grid_of(b, g), nt);
            LaunchEvents e;
            if (i == 0 && k == 0) e.start = ev.start;   // every group has sheet step 0
            if (i == last_g && k + 1 == m) e.stop = ev.stop;
            if (g.g->var[variant_of(b, g)].launch(md, grid, b->stream, sheet_descs(g, k), last ? g.d_last : g.d_tasks,
                                                  nt, g.d_ctrl, last ? 1 : b->tune.chunk, e))
                rc = set_err(LSR_EDEVICE, "persistent kernel launch failed: %s", hipGetErrorString(hipGetLastError()));
        }
    }
    return rc;
}

// Graph kinds: GRAPH_MID holds `len` middle round trips (tiled state in and
// out); GRAPH_CALL a whole call of `len` trips: the first row pass (row-major
// state in), len - 1 middle trips, the last row pass (row-major state out).
enum : int { GRAPH_MID = 0, GRAPH_CALL = 1 };
static constexpr size_t kMaxGraphs = 8;

// Destroy every captured graph (after the ones in flight have finished: the
// task tables and descriptors they read may be replaced next).
static void drop_graphs(lsr_batch_s* b) {
    if (b->graphs.empty()) return;
    if (b->launched && b->stream) (void)hipStreamSynchronize(b->stream);
    for (auto& g : b->graphs) (void)hipGraphExecDestroy(g.exec);
    b->graphs.clear();
    b->launched = false;
}

static int launch_trip(lsr_batch_s* b, int mode, LaunchEvents ev);

// The graph of (kind, len), captured on the batch's private stream on first
// use.  Graphs read the descriptors and task tables from device memory, so a
// graph stays valid until the batch regroups or repacks (drop_graphs).
static int get_graph(lsr_batch_s* b, int kind, int len, hipGraphExec_t* out) {
    for (auto& g : b->graphs)
        if (g.kind == kind && g.len == len) {
            g.used = ++b->graph_clock;
            *out = g.exec;
            return LSR_OK;
        }
    if (b->graphs.size() >= kMaxGraphs) {
        // evict the least recently used graph once nothing is in flight
        if (b->launched) LSR_HIP(hipStreamSynchronize(b->stream));
        b->launched = false;
        size_t lru = 0;
        for (size_t i = 1; i < b->graphs.size(); ++i)
            if (b->graphs[i].used < b->graphs[lru].used) lru = i;
        (void)hipGraphExecDestroy(b->graphs[lru].exec);
        b->graphs.erase(b->graphs.begin() + (long)lru);
    }
    hipGraph_t gr = nullptr;
    LSR_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    int rc = LSR_OK;
    if (kind == GRAPH_CALL) {
        rc = launch_trip(b, ROW_FIRST, {});
        for (int t = 1; t < len && rc == LSR_OK; ++t) rc = launch_trip(b, ROW_MID, {});
        if (rc == LSR_OK) rc = launch_trip(b, ROW_LAST, {});
    } else {
        for (int t = 0; t < len && rc == LSR_OK; ++t) rc = launch_trip(b, ROW_MID, {});
    }
    const hipError_t e = hipStreamEndCapture(b->stream, &gr);
    if (rc != LSR_OK) {
        if (gr) (void)hipGraphDestroy(gr);
        return rc;
    }
    if (e != hipSuccess) return set_err(LSR_EDEVICE, "graph capture failed: %s", hipGetErrorString(e));
    hipGraphExec_t ex = nullptr;
    const hipError_t ie = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (ie != hipSuccess) return set_err(LSR_EDEVICE, "graph instantiate failed: %s", hipGetErrorString(ie));
    lsr_batch_s::Graph g;
    g.kind = kind;
    g.len = len;
    g.exec = ex;
    g.used = ++b->graph_clock;
    b->graphs.push_back(g);
    *out = ex;
    return LSR_OK;
}

static int graph_launch(lsr_batch_s* b, hipGraphExec_t ex) {
    if (hipGraphLaunch(ex, b->stream) != hipSuccess)
        return set_err(LSR_EDEVICE, "graph launch failed: %s", hipGetErrorString(hipGetLastError()));
    b->launched = true;
    return LSR_OK;
}

// Per-cavity descriptors: refreshed when the state pointers change.
static int upload_descs(lsr_batch_s* b, void* const* E, void* const* N, bool force) {
    bool same = !force && b->lastE.size() == b->plans.size();
    for (size_t i = 0; same && i < b->plans.size(); ++i)
        same = b->lastE[i] == E[i] && b->lastN[i] == N[i] && b->lastVer[i] == b->plans[i]->version;
    if (same) return LSR_OK;
    for (auto& g : b->grp) {
        std::vector<CavDesc> h;
        for (int k = 0; k < g.sheets; ++k)
        for (int c : g.cav) {
            CavDesc d = plan_sheet_desc(b->plans[c], E[c], N[c], k);
            // only sheet 0's column pass folds the trip's sums into the trace
            if (k > 0) d.trace = nullptr;
            // the roughness kernels read d.rough without a check; a group runs
            // only the local-step codes it was compiled for
            if (((d.model & MODEL_ROUGH) != 0) != (d.rough != nullptr))
                return set_err(LSR_EINVAL, "cavity %d: roughness code and table disagree", c);
            const int lvl = g.g->any_model;
            const bool runs = lvl >= ANY_FIXED ? d.model == lvl - ANY_FIXED
                            : lvl == 2 ? true : lvl == 1 ? (d.model & MODEL_ROUGH) == 0 : d.model == 0;
            if (!runs) return set_err(LSR_EINVAL, "cavity %d: local-step code %d not in its group", c, d.model);
            if (d.prop_kind == 2 && (lvl != 1 && lvl != 2))
                return set_err(LSR_EINVAL, "cavity %d: general transfer function not in its group", c);
            if ((d.prop_kind == 2) != (d.trans != nullptr))
                return set_err(LSR_EINVAL, "cavity %d: propagator kind and transfer table disagree", c);
            for (int z = 0; z < g.g->nsizes; ++z)
                if (g.g->sizes[z] == d.N) d.tw = g.d_tw[z];
            d.nrb = group_blocks(g, d.N);
            h.push_back(d);
        }
        LSR_HIP(hipMemcpyAsync(g.d_desc, h.data(), h.size() * sizeof(CavDesc), hipMemcpyHostToDevice, b->stream));
        LSR_HIP(hipStreamSynchronize(b->stream));
    }
    b->lastE.assign(E, E + b->plans.size());
    b->lastN.assign(N, N + b->plans.size());
    b->lastVer.clear();
    for (auto* p : b->plans) b->lastVer.push_back(p->version);
    return LSR_OK;
}

// A plan's local-step code (model, roughness) or its general transfer
// function changed since the batch was grouped: regroup (the kernels of a
// group read the codes it was built for).
static int regroup_if_models_changed(lsr_batch_s* b) {
    bool same = b->models.size() == b->plans.size();
    for (size_t i = 0; same && i < b->plans.size(); ++i) same = b->models[i] == group_code(b->plans[i]);
    if (same) return LSR_OK;
    LSR_HIP(hipStreamSynchronize(b->stream));
    drop_graphs(b);
    return batch_partition(b);
}

// The launches of a call of n >= 1 trips.  With graphs (graph_k = k > 0): a
// call of n <= k + 1 trips replays one graph of the whole call; a longer call
// runs its first row pass, (n - 1) / k graphs of k trips, one graph of the
// remaining trips and its last row pass.  prepare_only captures and
// instantiates the graphs without launching anything.
static int run_trips(lsr_batch_s* b, int n, bool prepare_only = false) {
    const int k = b->tune.graph_k;
    hipGraphExec_t ex = nullptr;
    if (k <= 0) {
        if (prepare_only) return LSR_OK;
        int rc = launch_trip(b, ROW_FIRST, {});
        for (int t = 1; t < n && rc == LSR_OK; ++t) rc = launch_trip(b, ROW_MID, {});
        if (rc == LSR_OK) rc = launch_trip(b, ROW_LAST, {});
        return rc;
    }
    if (n - 1 <= k) {
        int rc = get_graph(b, GRAPH_CALL, n, &ex);
        return rc != LSR_OK || prepare_only ? rc : graph_launch(b, ex);
    }
    const int q = (n - 1) / k, r = (n - 1) % k;
    hipGraphExec_t ek = nullptr, er = nullptr;
    int rc = get_graph(b, GRAPH_MID, k, &ek);
    if (rc == LSR_OK && r > 0) rc = get_graph(b, GRAPH_MID, r, &er);
    if (rc != LSR_OK || prepare_only) return rc;
    rc = launch_trip(b, ROW_FIRST, {});
    for (int i = 0; i < q && rc == LSR_OK; ++i) rc = graph_launch(b, ek);
    if (rc == LSR_OK && r > 0) rc = graph_launch(b, er);
    if (rc == LSR_OK) rc = launch_trip(b, ROW_LAST, {});
    return rc;
}

// A batch orders its work after the caller's work on the stream its plans
// share, and the plans' own synchronising calls (lsr_sync, lsr_trace, the
// table-replacing setters) wait on that stream: every plan must be bound to
// the same stream, also after lsr_plan_set_stream.
static int check_streams(lsr_batch_s* b) {
    for (size_t i = 1; i < b->plans.size(); ++i)
        if (b->plans[i]->stream != b->plans[0]->stream)
            return set_err(LSR_EINVAL, "plan %zu is bound to another stream than plan 0", i);
    b->user = b->plans[0]->stream;
    return LSR_OK;
}

extern "C" {

int lsr_pack_tasks(const int* sizes, int count, int lag, int* tasks, int capacity) {
    if (!sizes || count < 1) return set_err(LSR_EINVAL, "no sizes");
    std::vector<int> nrb;
    for (int i = 0; i < count; ++i) {
        const int r = row_blocks(sizes[i]);
        if (!r) return set_err(LSR_EUNSUPPORTED, "N=%d is not compiled in", sizes[i]);
        nrb.push_back(r);
    }
    std::vector<int4> t;
    pack(nrb, lag >= 0 ? lag : default_lag(), true, t);
    if (!tasks) return (int)t.size();
    if (capacity < (int)t.size()) return set_err(LSR_EINVAL, "capacity %d < %zu tasks", capacity, t.size());
    for (size_t i = 0; i < t.size(); ++i) {
        tasks[3 * i] = t[i].x;
        tasks[3 * i + 1] = t[i].y;
        tasks[3 * i + 2] = t[i].z;
    }
    return (int)t.size();
}

int lsr_batch_create(lsr_batch* out, const lsr_plan* plans, int count) {
    if (!out) return set_err(LSR_EINVAL, "out is NULL");
    *out = nullptr;
    if (!plans || count < 1) return set_err(LSR_EINVAL, "a batch needs at least one plan");
    for (int i = 0; i < count; ++i) {
        if (!plans[i]) return set_err(LSR_EINVAL, "plan %d is NULL", i);
        if (plans[i]->prec != PREC_FP64TAB)
            return set_err(LSR_EUNSUPPORTED, "only FP64TAB plans (FP32 field, FP64-built tables) can be batched");
        if (plans[i]->device != plans[0]->device) return set_err(LSR_EINVAL, "plans on different devices");
        for (int j = 0; j < i; ++j)
            if (plans[j] == plans[i]) return set_err(LSR_EINVAL, "plan %d appears twice", i);
        if (plans[i]->stream != plans[0]->stream)
            return set_err(LSR_EINVAL, "plan %d is bound to another stream than plan 0", i);
    }
    lsr_batch_s* b = new (std::nothrow) lsr_batch_s();
    if (!b) return set_err(LSR_ENOMEM, "host allocation failed");
    b->device = plans[0]->device;
    DeviceGuard dg(b->device);
    b->plans.assign(plans, plans + count);
    b->user = plans[0]->stream;
    auto fail = [&](int rc) {
        batch_free(b);
        delete b;
        return rc;
    };
    if (hipDeviceGetAttribute(&b->cus, hipDeviceAttributeMultiprocessorCount, b->device) != hipSuccess)
        b->cus = 256;
    if (hipStreamCreateWithFlags(&b->stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) != hipSuccess)
        return fail(set_err(LSR_EDEVICE, "stream/event creation failed"));
    b->key = batch_key(b->plans);
    auto cache = cache_read(cache_path(nullptr));
    auto it = cache.find(b->key);
    if (it != cache.end()) b->tune = it->second;
    const int rc = batch_partition(b);
    if (rc) return fail(rc);
    *out = b;
    return LSR_OK;
}

int lsr_batch_set_graph_trips(lsr_batch b, int k) {
    if (!b || k < 0) return set_err(LSR_EINVAL, "bad batch or k");
    if (k != b->tune.graph_k) {
        DeviceGuard dg(b->device);
        drop_graphs(b);
        b->tune.graph_k = k;
    }
    return LSR_OK;
}

int lsr_batch_prepare(lsr_batch b, int n_trips) {
    if (!b || n_trips < 0) return set_err(LSR_EINVAL, "bad batch or n_trips");
    if (n_trips == 0) return LSR_OK;
    DeviceGuard dg(b->device);
    int rc = regroup_if_models_changed(b);
    if (rc == LSR_OK) rc = run_trips(b, n_trips, true);
    return rc;
}

int lsr_batch_test_wait(lsr_batch b, int extra_need, int spin_limit) {
    if (!b || extra_need < 0 || spin_limit < 0) return set_err(LSR_EINVAL, "bad batch or test setting");
    DeviceGuard dg(b->device);
    LSR_HIP(hipStreamSynchronize(b->stream));
    const unsigned w[2] = {(unsigned)spin_limit, (unsigned)extra_need};
    static_assert(CTRL_EXTRA == CTRL_SPIN + 1, "adjacent control words");
    for (auto& g : b->grp) LSR_HIP(hipMemcpy(g.d_ctrl + CTRL_SPIN, w, sizeof w, hipMemcpyHostToDevice));
    return LSR_OK;
}

int lsr_batch_configure(lsr_batch b, int engine, int variant, int wgs_per_cu, int chunk, int lag, int graph_k,
                        int merge, int shape, int* cfg_out) {
    if (!b) return set_err(LSR_EINVAL, "batch is NULL");
    if (engine > 2 || variant > 3 || chunk == 0 || chunk > 1024 || merge > 1 || shape > LSR_MAX_SHAPES)
        return set_err(LSR_EINVAL, "bad batch configuration");
    DeviceGuard dg(b->device);
    Tune t = b->tune;
    if (engine >= 0) t.engine = engine;
    if (variant >= 0) t.variant = variant;
    if (wgs_per_cu >= 0) t.wgs_per_cu = wgs_per_cu;
    if (chunk > 0) t.chunk = chunk;
    if (lag >= 0) t.lag = lag;
    if (graph_k >= 0) t.graph_k = graph_k;
    if (merge >= 0) t.merge = merge;
    if (shape >= 0) t.shape = shape;
    const bool regroup = t.merge != b->tune.merge || t.shape != b->tune.shape;
    const bool repack = t.lag != b->tune.lag;
    drop_graphs(b);
    b->tune = t;
    if (regroup || repack) {
        LSR_HIP(hipStreamSynchronize(b->stream));
        const int rc = regroup ? batch_partition(b) : batch_pack(b);
        if (rc) return rc;
    }
    if (cfg_out) {
        cfg_out[0] = t.engine;
        cfg_out[1] = t.variant;
        cfg_out[2] = t.wgs_per_cu;
        cfg_out[3] = t.chunk;
        cfg_out[4] = t.lag >= 0 ? t.lag : default_lag();
        cfg_out[5] = t.graph_k;
        cfg_out[6] = t.merge;
        cfg_out[7] = t.shape;
    }
    return LSR_OK;
}

int lsr_batch_roundtrips(lsr_batch b, void* const* E, void* const* N, int n_trips) {
    if (!b) return set_err(LSR_EINVAL, "batch is NULL");
    if (n_trips < 0) return set_err(LSR_EINVAL, "n_trips < 0");
    if (!E || !N) return set_err(LSR_EINVAL, "E or Ninv array is NULL");
    for (size_t i = 0; i < b->plans.size(); ++i) {
        if (!E[i] || !N[i] || ((uintptr_t)E[i] & 15u) || ((uintptr_t)N[i] & 15u))
            return set_err(LSR_EINVAL, "state %zu: NULL or not 16-byte aligned", i);
    }
    if (check_streams(b)) return LSR_EINVAL;
    if (n_trips == 0) return LSR_OK;
    DeviceGuard dg(b->device);
    // order after the caller's work on the plans' stream, and back
    LSR_HIP(hipEventRecord(b->ev_in, b->user));
    LSR_HIP(hipStreamWaitEvent(b->stream, b->ev_in, 0));
    int rc = regroup_if_models_changed(b);
    if (rc == LSR_OK) rc = upload_descs(b, E, N, false);
    if (rc == LSR_OK) rc = run_trips(b, n_trips);
    LSR_HIP(hipEventRecord(b->ev_out, b->stream));
    LSR_HIP(hipStreamWaitEvent(b->user, b->ev_out, 0));
    if (rc) return rc;
    for (auto* p : b->plans) {
        p->trips_done += (unsigned long long)n_trips;
        p->last_n = n_trips;
    }
    return LSR_OK;
}

int lsr_batch_time_kernels(lsr_batch b, void* const* E, void* const* N, int n_trips, double* ms) {
    if (!b || !ms || !E || !N) return set_err(LSR_EINVAL, "bad arguments");
    if (n_trips < 1) return set_err(LSR_EINVAL, "n_trips < 1");
    if (check_streams(b)) return LSR_EINVAL;
    DeviceGuard dg(b->device);
    LSR_HIP(hipEventRecord(b->ev_in, b->user));
    LSR_HIP(hipStreamWaitEvent(b->stream, b->ev_in, 0));
    int rc = regroup_if_models_changed(b);
    if (rc == LSR_OK) rc = upload_descs(b, E, N, false);
    if (rc) return rc;
    // dispatch timestamps of sheet step k of trip t (m steps per trip): row
    // pass (or the persistent kernels of the whole trip) start/stop = events
    // 4 (m t + k) + 0, 1; column pass start/stop = 4 (m t + k) + 2, 3
    const int m = max_sheets(b);
    const size_t ne = 4 * (size_t)m * (size_t)(n_trips + 1);
    std::vector<hipEvent_t> ev(ne, nullptr);
    auto at = [&](int t, int k, int j) { return ev[4 * ((size_t)m * t + k) + j]; };
    for (auto& e : ev)
        if (hipEventCreate(&e) != hipSuccess) {
            for (auto& x : ev)
                if (x) (void)hipEventDestroy(x);
            return set_err(LSR_EDEVICE, "hipEventCreate failed");
        }
    const bool grouped = b->tune.engine >= 1;
    for (int t = 0; t <= n_trips && rc == LSR_OK; ++t) {
        const int mode = t == 0 ? ROW_FIRST : (t == n_trips ? ROW_LAST : ROW_MID);
        if (grouped) {
            // the last row pass of a call is sheet 0's alone
            for (int k = 0; k < (mode == ROW_LAST ? 1 : m) && rc == LSR_OK; ++k) {
                const int md = k == 0 ? mode : ROW_MID;
                rc = launch_grouped_pass(b, md, TASK_ROW, LaunchEvents{at(t, k, 0), at(t, k, 1)}, k);
                if (rc == LSR_OK && md != ROW_LAST)
                    rc = launch_grouped_pass(b, md, TASK_COL, LaunchEvents{at(t, k, 2), at(t, k, 3)}, k);
            }
        } else {
            rc = launch_trip(b, mode, LaunchEvents{at(t, 0, 0), at(t, 0, 1)});
        }
    }
    double row = 0, col = 0, trip = 0;
    int nrow = 0;
    if (rc == LSR_OK && hipStreamSynchronize(b->stream) == hipSuccess) {
        for (int t = 0; t < n_trips; ++t) {
            if (n_trips > 1 && t == 0) continue;   // the FIRST form differs
            for (int k = 0; k < (grouped ? m : 1); ++k) {
                float a = 0, c = 0;
                (void)hipEventElapsedTime(&a, at(t, k, 0), at(t, k, 1));
                if (grouped) (void)hipEventElapsedTime(&c, at(t, k, 2), at(t, k, 3));
                row += a;
                col += c;
            }
            float w = 0;
            (void)hipEventElapsedTime(&w, at(t, 0, 0), at(t + 1, 0, 0));
            trip += w;
            ++nrow;
        }
    }
    for (auto& x : ev) (void)hipEventDestroy(x);
    LSR_HIP(hipEventRecord(b->ev_out, b->stream));
    LSR_HIP(hipStreamWaitEvent(b->user, b->ev_out, 0));
    if (rc) return rc;
    ms[0] = nrow ? row / nrow : 0;
    ms[1] = grouped && nrow ? col / nrow : 0;
    ms[2] = nrow ? trip / nrow : 0;
    for (auto* p : b->plans) {
        p->trips_done += (unsigned long long)n_trips;
        p->last_n = n_trips;
    }
    return LSR_OK;
}

int lsr_batch_diag(lsr_batch b, int idx, const void* E, const void* Ninv, lsr_diag_out* out) {
    if (!b || idx < 0 || idx >= (int)b->plans.size()) return set_err(LSR_EINVAL, "bad batch or index");
    return lsr_diag(b->plans[idx], E, Ninv, out);
}

void lsr_batch_destroy(lsr_batch b) {
    if (!b) return;
    DeviceGuard dg(b->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    batch_free(b);
    delete b;
}

// Time `trips` persistent trips (graph or eager per the tuning) on scratch
// state; returns ms per trip or a negative status.
static double time_batch(lsr_batch_s* b, const std::vector<void*>& E, const std::vector<void*>& N, int trips) {
    // no groups (a regrouping or repacking failed): nothing would run
    if (b->grp.empty()) return -1;
    if (upload_descs(b, E.data(), N.data(), false)) return -1;
    // warm-up with the timed call's length: its graphs are captured here,
    // outside the timing
    if (run_trips(b, trips)) return -1;
    hipEvent_t t0, t1;
    if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess) return -1;
    (void)hipEventRecord(t0, b->stream);
    const int rc = run_trips(b, trips);
    (void)hipEventRecord(t1, b->stream);
    float ms = -1;
    if (rc == 0 && hipEventSynchronize(t1) == hipSuccess) (void)hipEventElapsedTime(&ms, t0, t1);
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    return rc == 0 ? ms / trips : -1;
}

// One-cavity FFT plan of a plan alone: the cached choice for its size and
// precision form, else the fastest compiled one, timed over 200 trips on
// zero scratch state (the kernels have no data-dependent paths) and stored.
static int tune_plan(lsr_plan p, const char* path) {
    const std::string key = "gfx950:plan:" + std::to_string(p->N) + ":" + std::to_string(p->prec);
    const std::string cp = cache_path(path);
    auto cache = cache_read(cp);
    auto it = cache.find(key);
    if (it != cache.end()) return lsr_plan_set_fft_plan(p, it->second.shape);
    std::vector<int> cands = {0};
    for (int k = 1; k <= 3; ++k)
        if (p->prec != PREC_FP64 && launchers_alt(p->N, k)) cands.push_back(k);
    DeviceGuard dg(p->device);
    LSR_HIP(hipStreamSynchronize(p->stream));
    const size_t pts = (size_t)p->N * p->N;
    void *E = nullptr, *Nv = nullptr;
    if (dev_malloc(&E, pts * 2 * p->real_bytes()) != hipSuccess ||
        dev_malloc(&Nv, pts * p->real_bytes() * (size_t)p->slices) != hipSuccess) {
        if (E) (void)hipFree(E);
        return set_err(LSR_ENOMEM, "autotune scratch allocation failed");
    }
    (void)hipMemset(E, 0, pts * 2 * p->real_bytes());
    (void)hipMemset(Nv, 0, pts * p->real_bytes() * (size_t)p->slices);
    hipEvent_t t0 = nullptr, t1 = nullptr;
    int best = -1, rc = LSR_OK;
    float best_ms = 1e30f;
    if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess) rc = set_err(LSR_EDEVICE, "hipEventCreate failed");
    for (int k : cands) {
        if (rc != LSR_OK) break;
        if ((rc = lsr_plan_set_fft_plan(p, k)) != LSR_OK) break;
        if ((rc = lsr_roundtrips(p, E, Nv, 20)) != LSR_OK) break;   // warm-up
        (void)hipEventRecord(t0, p->stream);
        if ((rc = lsr_roundtrips(p, E, Nv, 200)) != LSR_OK) break;
        (void)hipEventRecord(t1, p->stream);
        float ms = 0;
        if (hipEventSynchronize(t1) != hipSuccess || hipEventElapsedTime(&ms, t0, t1) != hipSuccess) {
            rc = set_err(LSR_EDEVICE, "autotune timing failed");
            break;
        }
        if (ms < best_ms) {
            best_ms = ms;
            best = k;
        }
    }
    (void)hipStreamSynchronize(p->stream);
    if (t0) (void)hipEventDestroy(t0);
    if (t1) (void)hipEventDestroy(t1);
    (void)hipFree(E);
    (void)hipFree(Nv);
    if (rc != LSR_OK) return rc;
    rc = lsr_plan_set_fft_plan(p, best);
    if (rc != LSR_OK || cp.empty()) return rc;
    Tune t;
    t.shape = best;
    cache[key] = t;
    if (!cache_write(cp, cache)) return set_err(LSR_EINVAL, "cannot write tune cache %s", cp.c_str());
    return LSR_OK;
}

int lsr_autotune(lsr_plan p, lsr_batch b, const char* path) {
    if (!p && !b) return set_err(LSR_EINVAL, "nothing to tune");
    if (p && !b) return tune_plan(p, path);
    DeviceGuard dg(b->device);
    LSR_HIP(hipStreamSynchronize(b->user));
    // scratch state: zero fields (the kernels have no data-dependent paths)
    std::vector<void*> E, N;
    auto release = [&]() {
        for (void* x : E) (void)hipFree(x);
        for (void* x : N) (void)hipFree(x);
    };
    for (auto* q : b->plans) {
        void *e = nullptr, *n = nullptr;
        const size_t pts = (size_t)q->N * q->N;
        if (dev_malloc(&e, pts * 8) != hipSuccess || dev_malloc(&n, pts * 4) != hipSuccess) {
            if (e) (void)hipFree(e);
            release();
            return set_err(LSR_ENOMEM, "autotune scratch allocation failed");
        }
        (void)hipMemset(e, 0, pts * 8);
        (void)hipMemset(n, 0, pts * 4);
        E.push_back(e);
        N.push_back(n);
    }
    const Tune saved = b->tune;
    Tune best = saved;
    double best_ms = 1e30;
    long pts_total = 0;
    for (auto* q : b->plans) pts_total += (long)q->N * q->N;
    const int trips = pts_total > 32L * 1024 * 1024 ? 20 : 40;
    // merged grouping is a distinct choice only when some workgroup size
    // holds several grid sizes
    std::map<int, std::map<int, int>> by_threads;
    for (auto* q : b->plans) {
        ShapeInfo sh;
        shape_for(q->N, false, &sh);
        by_threads[sh.threads][q->N]++;
    }
    bool mixed = false;
    for (auto& kv : by_threads) mixed |= kv.second.size() > 1;
    auto consider = [&](const Tune& t, int n) {
        b->tune = t;
        drop_graphs(b);
        if (batch_pack(b)) return;
        const double ms = time_batch(b, E, N, n);
        if (ms > 0 && ms < best_ms) {
            best_ms = ms;
            best = b->tune;
        }
    };
    // alternative FFT plans compiled for some size of the batch
    int max_alt = 0;
    for (int gi = 0; gi < group_count(); ++gi) {
        const GroupInfo* g = group_at(gi);
        if (g->alt == 0 || g->nsizes != 1) continue;
        for (auto* q : b->plans)
            if (q->N == g->sizes[0]) max_alt = std::max(max_alt, g->alt);
    }
    for (int mg = 0; mg <= (mixed ? 1 : 0); ++mg)
    for (int sh = 0; sh <= (mg ? 0 : max_alt); ++sh) {
        b->tune = saved;
        b->tune.merge = mg;
        b->tune.shape = sh;
        if (batch_partition(b)) continue;
        const Tune base = b->tune;
        int nvar = 1;
        for (auto& g : b->grp) nvar = std::max(nvar, g.g->nvariants);
        // grouped launches, plain and software-pipelined: the register budget
        // is the only other choice
        for (int eng : {2, 1})
            for (int v = 0; v < nvar; ++v) {
                Tune t = base;
                t.engine = eng;
                t.variant = v;
                t.graph_k = 16;
                consider(t, trips);
            }
        // persistent-kernel settings for the default plans only
        for (int v = 0; v < (sh == 0 ? nvar : 0); ++v) {
            int occ = 1;
            for (auto& g : b->grp) occ = std::max(occ, g.occ[v < g.g->nvariants ? v : 0]);
            std::vector<int> wgs;
            for (int w = occ; w >= 1 && (int)wgs.size() < 3; --w) wgs.push_back(w);
            for (int w : wgs)
                for (int chunk : {1, 2, 4, 8})
                    for (int lag : {512, 2048, 8192}) {
                        Tune t = base;
                        t.engine = 0;
                        t.variant = v;
                        t.wgs_per_cu = w;
                        t.chunk = chunk;
                        t.lag = lag;
                        t.graph_k = 16;
                        consider(t, trips);
                    }
        }
    }
    if (best.merge != b->tune.merge || best.shape != b->tune.shape) {
        b->tune = best;
        if (batch_partition(b)) {
            release();
            return set_err(LSR_EDEVICE, "autotune: regrouping failed");
        }
    }
    for (int k : {0, 4, 16, 64}) {
        b->tune = best;
        b->tune.graph_k = k;
        drop_graphs(b);
        if (batch_pack(b)) continue;
        const double ms = time_batch(b, E, N, std::max(trips, k));
        if (ms > 0 && ms < best_ms * 0.995) {
            best_ms = ms;
            best = b->tune;
        }
    }
    (void)hipStreamSynchronize(b->stream);
    release();
    b->tune = best;
    drop_graphs(b);
    b->lastE.clear();
    b->lastN.clear();
    int rc = batch_pack(b);
    if (rc) return rc;
    if (best_ms >= 1e30) return set_err(LSR_EDEVICE, "autotune: no candidate ran");
    const std::string cp = cache_path(path);
    if (!cp.empty()) {
        auto cache = cache_read(cp);
        cache[b->key] = best;
        if (!cache_write(cp, cache)) return set_err(LSR_EINVAL, "cannot write tune cache %s", cp.c_str());
    }
    return LSR_OK;
}

}  // extern "C"
