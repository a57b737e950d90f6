// batch.cpp -- the batched form: many independent grids per call.
//
// Grids are grouped into classes by dimension, radius and size (2D grids of
// at least 2^18 cells and 3D grids of at least 2^20 cells are "large"), and
// optionally row alignment (row-aligned grids can use 128-bit accesses, but
// a class of their own makes for more, emptier pass rounds; measured on the
// 256-grid workload, joining them to the unaligned class is 7 % faster).  Every class has one kernel configuration -- temporal degree K
// and segment length, and for 3D lanes per row, cells per lane and
// wavefronts per workgroup -- taken from a tune override, the tuning cache
// or defaults, or measured on the batch's own grids by
// stencil_batch_autotune.
//
// A class runs as a chain of pass rounds.  Round p applies pass p of every
// grid of the class (K fused steps; a grid's last pass takes the remainder),
// ping-ponging between the grid's output and its plan's scratch so that the
// grid's last pass writes the output.  One round is one launch of the
// persistent work-list kernel of the class (one per distinct K in the
// round).  Chains are independent: they run on side streams forked from the
// origin stream and joined back into it.  The whole schedule is captured
// once into a HIP graph and replayed by every launch.  Because each item is
// computed by the same device code as the single-grid kernels, in the same
// operation order, every grid's output is bitwise that of stencil_run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "batch.hpp"
#include "launch.hpp"
#include "lowp.hpp"
#include "plan.hpp"
#include "stencil.h"

using namespace star;

namespace {

constexpr int64_t kLarge2D = (int64_t)1 << 18;
constexpr int64_t kLarge3D = (int64_t)1 << 20;
constexpr int kDefaultStreams = 4;
constexpr int kMaxStreams = 16;
constexpr int kOneShotCache = 4;

int bfail(int status, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return star_set_error(status, buf);
}

int bhip(hipError_t e, const char *what) {
    (void)hipGetLastError();
    return bfail(STENCIL_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

struct ClassCfg {
    int K = 1;
    int seg = 64;  // ly (2D) or lz (3D)
    int wl = 32, vec = 4, nw = 16;
};

struct BClass {
    int ndim = 2, R = 1;
    bool aligned = false;
    bool large = false;
    std::vector<int> grids;
    ClassCfg cfg;
    std::string tuned_by = "default";
    double gcells = 0.0;  // measured rate of the chain (autotune)
};

// Options of the tune string: per-dimension configuration overrides and the
// number of side streams.  0 = not given.
struct Options {
    int k2 = 0, ly = 0;
    int k3 = 0, wl = 0, vec = 0, nw = 0, lz = 0;
    int streams = 0;
    int graph = -1;
    int merge = -1;  // 0: row-aligned grids keep classes of their own (default: they join
                     // the unaligned class of their kind -- fewer, fuller pass rounds)
};

struct Launch {
    BatchLaunchArgs a;
    int chain;
    size_t entry_off;
};

// Classes whose configurations select the same kernel (dimension, radius,
// alignment, K and for 3D vec/wl/nw) share one chain: their grids run in
// the same launches, each grid with its own class's segment length.
struct Sched {
    std::vector<BatchGrid> grids;     // one per batch grid (unused slots stay zero)
    std::vector<BatchEntry> entries;
    std::vector<Launch> launches;     // chain-major, rounds in order
    std::vector<std::vector<int>> chains;  // class ids per chain
    std::vector<int> chain_begin, chain_end;
    std::vector<int> chain_of_class;
};

struct DevTables {
    BatchGrid *grids = nullptr;
    BatchEntry *entries = nullptr;
    unsigned *counters = nullptr;
    void release() {
        if (grids || entries || counters) (void)hipDeviceSynchronize();
        if (grids) (void)hipFree(grids);
        if (entries) (void)hipFree(entries);
        if (counters) (void)hipFree(counters);
        grids = nullptr;
        entries = nullptr;
        counters = nullptr;
    }
};

int kmax(int ndim, int R) { return ndim == 2 ? max_k2d(R) : max_k3d(R); }

std::string class_name(const BClass &c) {
    char buf[64];
    snprintf(buf, sizeof buf, "%dd r=%d al=%d %s", c.ndim, c.R, c.aligned ? 1 : 0,
             c.large ? "large" : "small");
    return buf;
}

std::string cfg_string(const BClass &c, const ClassCfg &g) {
    char buf[96];
    if (c.ndim == 2)
        snprintf(buf, sizeof buf, "k=%d,ly=%d", g.K, g.seg);
    else
        snprintf(buf, sizeof buf, "k=%d,wl=%d,vec=%d,nw=%d,lz=%d", g.K, g.wl, g.vec, g.nw, g.seg);
    return buf;
}

std::string cache_key(const BClass &c, int device) {
    char buf[128];
    snprintf(buf, sizeof buf, "batch ndim=%d R=%d aligned=%d size=%s arch=%s", c.ndim, c.R,
             c.aligned ? 1 : 0, c.large ? "large" : "small", tune_arch_name(device).c_str());
    return buf;
}

size_t lds3d(const ClassCfg &g, int K) {
    return (size_t)K * 2 * g.nw * (64 / g.wl) * g.wl * g.vec * sizeof(float) + 16;
}

bool cfg_valid(const BClass &c, const ClassCfg &g) {
    if (g.K < 1 || g.K > kmax(c.ndim, c.R) || g.seg < 1) return false;
    if (c.ndim == 2) return true;
    if (g.wl != 32 && g.wl != 64) return false;
    if (!(g.vec == 4 || (g.vec == 8 && g.wl == 64 && vec8_ok(c.R, g.K, c.aligned)))) return false;
    if (g.nw < 1 || g.nw > 16 || g.nw * (64 / g.wl) <= 2 * g.K * c.R) return false;
    return lds3d(g, g.K) <= 160 * 1024;
}

ClassCfg default_cfg(const BClass &c) {
    ClassCfg g;
    if (c.ndim == 2) {
        static const int k2[4] = {8, 5, 4, 4};
        g.K = std::min(k2[c.R - 1], max_k2d(c.R));
        g.seg = c.large ? 128 : 64;
    } else {
        g.K = c.R == 1 ? 4 : c.R == 2 ? 2 : 1;
        g.wl = 32;
        g.vec = 4;
        g.nw = 16;
        g.seg = c.large ? 64 : 16;
    }
    return g;
}

bool parse_int(const std::string &s, int *out) {
    char *end = nullptr;
    const long v = strtol(s.c_str(), &end, 10);
    if (s.empty() || *end != '\0' || v < 0 || v > (1 << 30)) return false;
    *out = (int)v;
    return true;
}

// Parses "k=..,ly=.." (2D) or "k=..,wl=..,vec=..,nw=..,lz=.." (3D).
bool parse_cfg(const BClass &c, const std::string &s, ClassCfg *g) {
    ClassCfg r = default_cfg(c);
    size_t pos = 0;
    while (pos <= s.size()) {
        size_t comma = s.find(',', pos);
        if (comma == std::string::npos) comma = s.size();
        const std::string item = s.substr(pos, comma - pos);
        pos = comma + 1;
        if (item.empty()) continue;
        const size_t eq = item.find('=');
        int v = 0;
        if (eq == std::string::npos || !parse_int(item.substr(eq + 1), &v)) return false;
        const std::string key = item.substr(0, eq);
        if (key == "k") r.K = v;
        else if (key == "ly" && c.ndim == 2) r.seg = v;
        else if (key == "lz" && c.ndim == 3) r.seg = v;
        else if (key == "wl" && c.ndim == 3) r.wl = v;
        else if (key == "vec" && c.ndim == 3) r.vec = v;
        else if (key == "nw" && c.ndim == 3) r.nw = v;
        else return false;
    }
    if (!cfg_valid(c, r)) return false;
    *g = r;
    return true;
}

int parse_options(const char *tune, Options *o) {
    if (!tune) return STENCIL_OK;
    const std::string s(tune);
    size_t pos = 0;
    while (pos <= s.size()) {
        size_t comma = s.find(',', pos);
        if (comma == std::string::npos) comma = s.size();
        const std::string item = s.substr(pos, comma - pos);
        pos = comma + 1;
        if (item.empty()) continue;
        const size_t eq = item.find('=');
        int v = 0;
        if (eq == std::string::npos || !parse_int(item.substr(eq + 1), &v))
            return bfail(STENCIL_EINVAL, "bad batch tune item '%s'", item.c_str());
        const std::string key = item.substr(0, eq);
        const bool pos_ok = v >= 1;
        if (key == "2d.k" && pos_ok) o->k2 = v;
        else if (key == "2d.ly" && pos_ok) o->ly = v;
        else if (key == "3d.k" && pos_ok) o->k3 = v;
        else if (key == "3d.wl" && (v == 32 || v == 64)) o->wl = v;
        else if (key == "3d.vec" && (v == 4 || v == 8)) o->vec = v;
        else if (key == "3d.nw" && pos_ok && v <= 16) o->nw = v;
        else if (key == "3d.lz" && pos_ok) o->lz = v;
        else if (key == "streams" && v <= kMaxStreams) o->streams = v;
        else if (key == "graph" && v <= 1) o->graph = v;
        else if (key == "merge" && v <= 1) o->merge = v;
        else return bfail(STENCIL_EINVAL, "bad batch tune item '%s'", item.c_str());
    }
    return STENCIL_OK;
}

// Resident workgroups per CU of a launch's kernel (0 = not built).
int occupancy(int ndim, int R, const BatchLaunchArgs &a) {
    if (ndim == 2) {
        switch (R) {
            case 1: return batch2d_occupancy_r1(a);
            case 2: return batch2d_occupancy_r2(a);
            case 3: return batch2d_occupancy_r3(a);
            case 4: return batch2d_occupancy_r4(a);
        }
    } else {
        switch (R) {
            case 1: return batch3d_occupancy_r1(a);
            case 2: return batch3d_occupancy_r2(a);
            case 3: return batch3d_occupancy_r3(a);
            case 4: return batch3d_occupancy_r4(a);
        }
    }
    return 0;
}

hipError_t launch_one(int ndim, int R, const BatchLaunchArgs &a, hipStream_t s) {
    if (ndim == 2) {
        switch (R) {
            case 1: return launch_batch2d_r1(a, s);
            case 2: return launch_batch2d_r2(a, s);
            case 3: return launch_batch2d_r3(a, s);
            case 4: return launch_batch2d_r4(a, s);
        }
    } else {
        switch (R) {
            case 1: return launch_batch3d_r1(a, s);
            case 2: return launch_batch3d_r2(a, s);
            case 3: return launch_batch3d_r3(a, s);
            case 4: return launch_batch3d_r4(a, s);
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace

struct stencil_batch_s {
    int device = 0;
    int ncu = 256;
    int n = 0;
    std::vector<stencil_plan_t> plans;
    std::vector<const float *> ins;
    std::vector<float *> outs;
    std::vector<int64_t> steps;
    std::vector<int> own;            // grids run by their own plan: steps == 0 or not FP32 storage
    std::vector<BClass> classes;
    Options opt;
    int nstreams = kDefaultStreams;
    bool use_graph = true;

    Sched sched;
    DevTables tabs;
    std::vector<int> stream_of_chain;
    std::vector<hipStream_t> side;
    hipStream_t cap = nullptr;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> join;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;

    ~stencil_batch_s() {
        if (exec || graph || cap || !side.empty()) (void)hipDeviceSynchronize();
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        tabs.release();
        for (hipStream_t s : side) (void)hipStreamDestroy(s);
        if (cap) (void)hipStreamDestroy(cap);
        if (fork) (void)hipEventDestroy(fork);
        for (hipEvent_t e : join) (void)hipEventDestroy(e);
    }
};

namespace {

// Steps of grid g fused per pass and its number of passes.
void grid_passes(const stencil_batch_s *b, int g, int K, int *np, int *tail) {
    const int64_t s = b->steps[g];
    const int64_t n = (s + K - 1) / K;
    *np = (int)n;
    *tail = (int)(s - (n - 1) * K);
}

// Groups classes into chains: classes with the same kernel share one.
std::vector<std::vector<int>> make_chains(const stencil_batch_s *b, const std::vector<int> &cls_ids) {
    std::map<std::tuple<int, int, int, int, int, int, int>, int> index;
    std::vector<std::vector<int>> chains;
    for (int c : cls_ids) {
        const BClass &C = b->classes[c];
        const ClassCfg &g = C.cfg;
        const bool d3 = C.ndim == 3;
        const auto key = std::make_tuple(C.ndim, C.R, C.aligned ? 1 : 0, g.K, d3 ? g.vec : 0,
                                         d3 ? g.wl : 0, d3 ? g.nw : 0);
        auto it = index.find(key);
        if (it == index.end()) {
            it = index.emplace(key, (int)chains.size()).first;
            chains.emplace_back();
        }
        chains[it->second].push_back(c);
    }
    return chains;
}

// Work-list schedule of the given chains.
int build_sched(const stencil_batch_s *b, const std::vector<std::vector<int>> &chains, Sched *out) {
    Sched s;
    s.grids.assign(b->n, BatchGrid{});
    s.chains = chains;
    s.chain_begin.assign(chains.size(), 0);
    s.chain_end.assign(chains.size(), 0);
    s.chain_of_class.assign(b->classes.size(), -1);
    for (size_t ch = 0; ch < chains.size(); ++ch) {
        const int c = chains[ch][0];
        for (int cc : chains[ch]) s.chain_of_class[cc] = (int)ch;
        const BClass &C = b->classes[c];
        const ClassCfg &g = C.cfg;
        const int R = C.R;
        s.chain_begin[ch] = (int)s.launches.size();
        std::vector<int> grids;
        for (int cc : chains[ch]) grids.insert(grids.end(), b->classes[cc].grids.begin(), b->classes[cc].grids.end());
        int P = 0;
        for (int cc : chains[ch])
            for (int gi : b->classes[cc].grids) {
                const stencil_plan_s *p = b->plans[gi];
                BatchGrid &bg = s.grids[gi];
                bg.cf = p->cf;
                bg.nx = (int)p->nx;
                bg.ny = (int)p->ny;
                bg.nz = (int)p->nz;
                bg.seg = (int)std::min<int64_t>(b->classes[cc].cfg.seg, C.ndim == 2 ? p->ny : p->nz);
            }
        for (int gi : grids) {
            int np = 0, tail = 0;
            grid_passes(b, gi, g.K, &np, &tail);
            P = std::max(P, np);
        }
        for (int round = 0; round < P; ++round) {
            std::map<int, std::vector<int>> by_k;
            for (int gi : grids) {
                int np = 0, tail = 0;
                grid_passes(b, gi, g.K, &np, &tail);
                if (round < np) by_k[round == np - 1 ? tail : g.K].push_back(gi);
            }
            for (auto &kv : by_k) {
                const int K = kv.first;
                BatchLaunchArgs a{};
                a.K = K;
                a.aligned = C.aligned;
                a.vec = (K == g.K) ? g.vec : 4;
                a.wl = g.wl;
                a.nw = g.nw;
                struct E {
                    BatchEntry e;
                    int64_t items;
                    int cost;
                };
                std::vector<E> es;
                for (int gi : kv.second) {
                    const stencil_plan_s *p = b->plans[gi];
                    const BatchGrid &bg = s.grids[gi];
                    int np = 0, tail = 0;
                    grid_passes(b, gi, g.K, &np, &tail);
                    E x{};
                    x.e.grid = gi;
                    const bool dst_out = ((np - 1 - round) % 2) == 0;
                    x.e.dst = dst_out ? b->outs[gi] : p->scratch;
                    x.e.src = round == 0 ? b->ins[gi] : (dst_out ? p->scratch : b->outs[gi]);
                    int64_t nseg;
                    if (C.ndim == 2) {
                        const int TX = star2d_tile_x(K, R);
                        x.e.ntx = (bg.nx + TX - 1) / TX;
                        x.e.nty = 1;
                        nseg = (bg.ny + bg.seg - 1) / bg.seg;
                        x.cost = std::min(bg.seg, bg.ny) + 2 * K * R;
                    } else {
                        const int W = a.wl * a.vec;
                        const int ty = a.nw * (64 / a.wl) - 2 * K * R;
                        if (bg.nx > W || a.wl != 64) {
                            x.e.hx = (K * R + a.vec - 1) / a.vec * a.vec;
                            x.e.tx = W - 2 * x.e.hx;
                            x.e.ntx = (bg.nx + x.e.tx - 1) / x.e.tx;
                        } else {
                            x.e.hx = 0;
                            x.e.tx = bg.nx;
                            x.e.ntx = 1;
                        }
                        x.e.nty = (bg.ny + ty - 1) / ty;
                        nseg = (bg.nz + bg.seg - 1) / bg.seg;
                        x.cost = std::min(bg.seg, bg.nz) + 2 * K * R;
                    }
                    x.items = (int64_t)x.e.ntx * x.e.nty * nseg;
                    es.push_back(x);
                }
                // longest items first: the counter deals them in entry order
                std::stable_sort(es.begin(), es.end(),
                                 [](const E &u, const E &v) { return u.cost > v.cost; });
                Launch L{};
                L.chain = (int)ch;
                L.entry_off = s.entries.size();
                int64_t item0 = 0;
                for (E &x : es) {
                    x.e.item0 = (int)item0;
                    item0 += x.items;
                    if (item0 > (int64_t)0x7fffffff)
                        return bfail(STENCIL_EUNSUPPORTED, "a pass round of the batch exceeds 2^31 work items");
                    s.entries.push_back(x.e);
                }
                a.nentries = (int)es.size();
                a.nitems = (int)item0;
                const int occ = occupancy(C.ndim, R, a);
                if (occ < 1)
                    return bfail(STENCIL_EUNSUPPORTED, "no work-list kernel for class %s with %s",
                                 class_name(C).c_str(), cfg_string(C, g).c_str());
                const int64_t per_block = C.ndim == 2 ? 4 : 1;
                const int64_t want = (a.nitems + per_block - 1) / per_block;
                a.blocks = (int)std::min<int64_t>(want, (int64_t)occ * b->ncu);
                L.a = a;
                s.launches.push_back(L);
            }
        }
        s.chain_end[ch] = (int)s.launches.size();
    }
    *out = std::move(s);
    return STENCIL_OK;
}

int upload(const Sched &s, DevTables *t) {
    t->release();
    const size_t ng = std::max<size_t>(1, s.grids.size());
    const size_t ne = std::max<size_t>(1, s.entries.size());
    const size_t nc = std::max<size_t>(1, s.launches.size());
    hipError_t e = hipMalloc(&t->grids, ng * sizeof(BatchGrid));
    if (e == hipSuccess) e = hipMalloc(&t->entries, ne * sizeof(BatchEntry));
    if (e == hipSuccess) e = hipMalloc(&t->counters, nc * sizeof(unsigned));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        t->release();
        return bfail(STENCIL_ENOMEM, "hipMalloc of the batch work lists failed");
    }
    if (!s.grids.empty())
        e = hipMemcpy(t->grids, s.grids.data(), s.grids.size() * sizeof(BatchGrid), hipMemcpyHostToDevice);
    if (e == hipSuccess && !s.entries.empty())
        e = hipMemcpy(t->entries, s.entries.data(), s.entries.size() * sizeof(BatchEntry),
                      hipMemcpyHostToDevice);
    if (e != hipSuccess) return bhip(e, "hipMemcpy of the batch work lists");
    return STENCIL_OK;
}

BatchLaunchArgs bind(const Launch &L, const DevTables &t, size_t li) {
    BatchLaunchArgs a = L.a;
    a.entries = t.entries + L.entry_off;
    a.grids = t.grids;
    a.counter = t.counters + li;
    return a;
}

// Enqueues the launches of one chain on `s`.
hipError_t enqueue_chain(const stencil_batch_s *b, const Sched &sc, const DevTables &t, int ch,
                         hipStream_t s) {
    const BClass &C = b->classes[sc.chains[ch][0]];
    for (int li = sc.chain_begin[ch]; li < sc.chain_end[ch]; ++li) {
        const hipError_t e = launch_one(C.ndim, C.R, bind(sc.launches[li], t, (size_t)li), s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Enqueues the whole batch on `origin`: counters cleared by a fill kernel,
// the grids run by their own plan, then every class chain on its side
// stream, joined back into `origin`.
hipError_t enqueue_all(const stencil_batch_s *b, hipStream_t origin) {
    hipError_t e = hipSuccess;
    if (!b->sched.launches.empty()) {
        e = lowp_fill_u32(b->tabs.counters, (int64_t)b->sched.launches.size(), 0u, origin);
        if (e != hipSuccess) return e;
    }
    for (int g : b->own) {
        e = plan_enqueue(b->plans[g], b->ins[g], b->outs[g], b->steps[g], origin);
        if (e != hipSuccess) return e;
    }
    const int nc = (int)b->sched.chains.size();
    if (nc == 0) return hipSuccess;
    if (b->side.empty()) {
        for (int c = 0; c < nc; ++c)
            if ((e = enqueue_chain(b, b->sched, b->tabs, c, origin)) != hipSuccess) return e;
        return hipSuccess;
    }
    if ((e = hipEventRecord(b->fork, origin)) != hipSuccess) return e;
    for (hipStream_t s : b->side)
        if ((e = hipStreamWaitEvent(s, b->fork, 0)) != hipSuccess) return e;
    for (int c = 0; c < nc; ++c)
        if ((e = enqueue_chain(b, b->sched, b->tabs, c, b->side[b->stream_of_chain[c]])) != hipSuccess)
            return e;
    for (size_t i = 0; i < b->side.size(); ++i) {
        if ((e = hipEventRecord(b->join[i], b->side[i])) != hipSuccess) return e;
        if ((e = hipStreamWaitEvent(origin, b->join[i], 0)) != hipSuccess) return e;
    }
    return hipSuccess;
}

// Spreads the chains over the side streams, longest first onto the least
// loaded stream.  A chain's cost is its classes' measured time when all were
// autotuned, else an estimate: cell-steps at 1 TCell/s plus 5 us per round.
void assign_streams(stencil_batch_s *b) {
    const Sched &sc = b->sched;
    const int nc = (int)sc.chains.size();
    std::vector<double> cost(nc, 0.0);
    for (int ch = 0; ch < nc; ++ch) {
        for (int c : sc.chains[ch]) {
            const BClass &C = b->classes[c];
            double cellsteps = 0.0;
            for (int g : C.grids) cellsteps += (double)b->plans[g]->ncells * (double)b->steps[g];
            cost[ch] += C.gcells > 0.0 ? cellsteps / (C.gcells * 1e6) : cellsteps * 1e-9;
        }
        cost[ch] += (sc.chain_end[ch] - sc.chain_begin[ch]) * 5e-3;
    }
    std::vector<int> order(nc);
    for (int c = 0; c < nc; ++c) order[c] = c;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return cost[x] > cost[y]; });
    const int S = std::max<int>(1, (int)b->side.size());
    std::vector<double> load(S, 0.0);
    b->stream_of_chain.assign(nc, 0);
    for (int c : order) {
        const int s = (int)(std::min_element(load.begin(), load.end()) - load.begin());
        b->stream_of_chain[c] = s;
        load[s] += cost[c];
    }
}

// (Re)builds the schedule and its device tables and captures the graph.
int batch_build(stencil_batch_s *b) {
    std::vector<int> all(b->classes.size());
    for (size_t c = 0; c < all.size(); ++c) all[c] = (int)c;
    Sched s;
    int rc = build_sched(b, make_chains(b, all), &s);
    if (rc != STENCIL_OK) return rc;
    if (b->exec) {
        (void)hipDeviceSynchronize();
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    if (b->graph) {
        (void)hipGraphDestroy(b->graph);
        b->graph = nullptr;
    }
    rc = upload(s, &b->tabs);
    if (rc != STENCIL_OK) return rc;
    b->sched = std::move(s);
    assign_streams(b);
    if (!b->use_graph) return STENCIL_OK;
    hipError_t e = hipStreamBeginCapture(b->cap, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return bhip(e, "hipStreamBeginCapture");
    const hipError_t eq = enqueue_all(b, b->cap);
    hipGraph_t g = nullptr;
    e = hipStreamEndCapture(b->cap, &g);
    if (eq != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return bhip(eq, "capture of the batch launches");
    }
    if (e != hipSuccess) return bhip(e, "hipStreamEndCapture");
    b->graph = g;
    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        b->exec = nullptr;
        return bhip(e, "hipGraphInstantiate");
    }
    return STENCIL_OK;
}

bool overlap(uintptr_t a, size_t na, uintptr_t b, size_t nb) { return a < b + nb && b < a + na; }

int batch_create(stencil_batch_t *out, int n, const stencil_plan_t *plans, const float *const *ins,
                 float *const *outs, const int64_t *steps, const char *tune) {
    if (!out) return bfail(STENCIL_EINVAL, "batch pointer is NULL");
    *out = nullptr;
    if (n < 1) return bfail(STENCIL_EINVAL, "a batch needs n >= 1 grids (got %d)", n);
    if (!plans || !ins || !outs || !steps) return bfail(STENCIL_EINVAL, "NULL batch array");
    Options opt;
    int rc = parse_options(tune, &opt);
    if (rc != STENCIL_OK) return rc;
    for (int g = 0; g < n; ++g) {
        rc = run_check(plans[g], ins[g], outs[g], steps[g]);
        if (rc != STENCIL_OK) {
            const std::string m = stencil_last_error();
            return bfail(rc, "grid %d: %s", g, m.c_str());
        }
        if (plans[g]->device != plans[0]->device)
            return bfail(STENCIL_EINVAL, "grid %d: plans of one batch must share a device", g);
    }
    // Grids run concurrently: a grid may not write memory another grid
    // reads or writes, and a plan (its scratch) may appear only once.
    {
        struct Rg {
            uintptr_t p;
            size_t n;
            int g;
            bool w;
        };
        std::vector<Rg> rg;
        for (int g = 0; g < n; ++g) {
            const size_t bytes = (size_t)plans[g]->ncells * sizeof(float);
            rg.push_back({(uintptr_t)ins[g], bytes, g, false});
            rg.push_back({(uintptr_t)outs[g], bytes, g, true});
            rg.push_back({(uintptr_t)plans[g]->scratch, bytes, g, true});
        }
        std::sort(rg.begin(), rg.end(), [](const Rg &x, const Rg &y) { return x.p < y.p; });
        for (size_t i = 0; i < rg.size(); ++i)
            for (size_t j = i + 1; j < rg.size() && rg[j].p < rg[i].p + rg[i].n; ++j)
                if (rg[i].g != rg[j].g && (rg[i].w || rg[j].w))
                    return bfail(STENCIL_EINVAL,
                                 "grids %d and %d overlap (a plan, output or scratch is shared)",
                                 rg[i].g, rg[j].g);
    }
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return bhip(e, "hipGetDevice");
    if (dev != plans[0]->device)
        return bfail(STENCIL_EINVAL, "the current device (%d) is not the plans' device (%d)", dev,
                     plans[0]->device);

    auto *b = new (std::nothrow) stencil_batch_s();
    if (!b) return bfail(STENCIL_ENOMEM, "host allocation failed");
    b->device = dev;
    b->n = n;
    b->opt = opt;
    b->plans.assign(plans, plans + n);
    b->ins.assign(ins, ins + n);
    b->outs.assign(outs, outs + n);
    b->steps.assign(steps, steps + n);
    b->use_graph = opt.graph != 0;
    if (hipDeviceGetAttribute(&b->ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        b->ncu < 1)
        b->ncu = 256;

    // classes
    std::map<std::tuple<int, int, int, int>, int> index;
    for (int g = 0; g < n; ++g) {
        const stencil_plan_s *p = plans[g];
        // rows (2D) and planes (3D) are addressed through buffer descriptors
        // whose byte sizes must stay below 2^31
        const bool wide_plane = (p->ndim == 3 && p->nx * p->ny * 4 >= ((int64_t)1 << 31)) ||
                                (p->ndim == 2 && p->nx * 4 >= ((int64_t)1 << 31));
        const bool high_radius = p->radius > 4;  // work-list kernels are built for R <= 4
        // ... and for per-point coefficients with the clamp boundary
        const bool other_form = p->pad != 0 || p->sym != 0;
        if (steps[g] == 0 || p->storage != STENCIL_F32 || wide_plane || high_radius || other_form) {
            b->own.push_back(g);
            continue;
        }
        const bool al = opt.merge == 0 && p->nx % 4 == 0 &&
                        ((((uintptr_t)ins[g]) | ((uintptr_t)outs[g]) | ((uintptr_t)p->scratch)) & 15) == 0;
        const bool large = p->ncells >= (p->ndim == 2 ? kLarge2D : kLarge3D);
        const auto key = std::make_tuple(p->ndim, p->radius, al ? 1 : 0, large ? 1 : 0);
        auto it = index.find(key);
        if (it == index.end()) {
            BClass c;
            c.ndim = p->ndim;
            c.R = p->radius;
            c.aligned = al;
            c.large = large;
            it = index.emplace(key, (int)b->classes.size()).first;
            b->classes.push_back(c);
        }
        b->classes[it->second].grids.push_back(g);
    }
    for (BClass &c : b->classes) {
        c.cfg = default_cfg(c);
        c.tuned_by = "default";
        std::string cached;
        ClassCfg g;
        if (tune_cache_get(cache_key(c, dev), cached) && parse_cfg(c, cached, &g)) {
            c.cfg = g;
            c.tuned_by = "cache";
        }
        const bool any = c.ndim == 2 ? (opt.k2 || opt.ly) : (opt.k3 || opt.wl || opt.vec || opt.nw || opt.lz);
        if (any) {
            // overrides: K is capped at the class's largest built K
            if (c.ndim == 2) {
                if (opt.k2) c.cfg.K = std::min(opt.k2, max_k2d(c.R));
                if (opt.ly) c.cfg.seg = opt.ly;
            } else {
                if (opt.k3) c.cfg.K = std::min(opt.k3, max_k3d(c.R));
                if (opt.wl) c.cfg.wl = opt.wl;
                if (opt.vec) c.cfg.vec = opt.vec;
                if (opt.nw) c.cfg.nw = opt.nw;
                if (opt.lz) c.cfg.seg = opt.lz;
                if (c.cfg.vec == 8 && !(c.cfg.wl == 64 && vec8_ok(c.R, c.cfg.K, c.aligned))) c.cfg.vec = 4;
            }
            c.tuned_by = "override";
        }
        if (!cfg_valid(c, c.cfg)) {
            const std::string name = class_name(c), cfg = cfg_string(c, c.cfg);
            delete b;
            return bfail(STENCIL_EINVAL, "configuration %s is not valid for class %s", cfg.c_str(),
                         name.c_str());
        }
    }
    // streams and events
    const int want = opt.streams ? opt.streams : kDefaultStreams;
    b->nstreams = std::min<int>(want, (int)b->classes.size());  // chains <= classes
    e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    for (int i = 0; e == hipSuccess && i < b->nstreams && b->nstreams > 1; ++i) {
        hipStream_t s = nullptr;
        hipEvent_t j = nullptr;
        e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
        if (e == hipSuccess) b->side.push_back(s);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&j, hipEventDisableTiming);
        if (e == hipSuccess) b->join.push_back(j);
    }
    if (e != hipSuccess) {
        delete b;
        return bhip(e, "stream/event creation");
    }
    rc = batch_build(b);
    if (rc != STENCIL_OK) {
        delete b;
        return rc;
    }
    *out = b;
    return STENCIL_OK;
}

// Candidate configurations of a class for the autotuner.
std::vector<ClassCfg> candidates(const stencil_batch_s *b, const BClass &c) {
    std::vector<ClassCfg> out;
    int64_t max_len = 1;
    for (int g : c.grids) max_len = std::max(max_len, c.ndim == 2 ? b->plans[g]->ny : b->plans[g]->nz);
    if (c.ndim == 2) {
        for (int K = 1; K <= max_k2d(c.R); ++K)
            for (int ly : {16, 32, 64, 128, 256}) {
                if (ly > max_len && ly != 16) continue;
                ClassCfg g;
                g.K = K;
                g.seg = ly;
                out.push_back(g);
            }
    } else {
        for (int K = 1; K <= max_k3d(c.R); ++K)
            for (int wl : {32, 64})
                for (int vec : {4, 8})
                    for (int nw : {8, 16})
                        for (int lz : {8, 16, 32, 64}) {
                            if (lz > max_len && lz != 8) continue;
                            ClassCfg g;
                            g.K = K;
                            g.wl = wl;
                            g.vec = vec;
                            g.nw = nw;
                            g.seg = lz;
                            if (cfg_valid(c, g)) out.push_back(g);
                        }
    }
    return out;
}

int batch_autotune(stencil_batch_s *b, std::string &report, hipStream_t st) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return bfail(STENCIL_EDEVICE, "hipEventCreate failed");
    int rc = STENCIL_OK;
    for (size_t ci = 0; ci < b->classes.size() && rc == STENCIL_OK; ++ci) {
        BClass &C = b->classes[ci];
        double cellsteps = 0.0;
        for (int g : C.grids) cellsteps += (double)b->plans[g]->ncells * (double)b->steps[g];
        const ClassCfg saved = C.cfg;
        ClassCfg best = saved;
        double best_rate = -1.0;
        for (const ClassCfg &cand : candidates(b, C)) {
            C.cfg = cand;
            Sched s;
            if (build_sched(b, {{(int)ci}}, &s) != STENCIL_OK) continue;
            DevTables t;
            if (upload(s, &t) != STENCIL_OK) {
                t.release();
                continue;
            }
            auto run = [&]() -> hipError_t {
                hipError_t e = lowp_fill_u32(t.counters, (int64_t)s.launches.size(), 0u, st);
                for (int li = s.chain_begin[0]; e == hipSuccess && li < s.chain_end[0]; ++li)
                    e = launch_one(C.ndim, C.R, bind(s.launches[li], t, (size_t)li), st);
                return e;
            };
            float ms = 0.0f;
            const bool ok = run() == hipSuccess && hipEventRecord(e0, st) == hipSuccess &&
                            run() == hipSuccess && hipEventRecord(e1, st) == hipSuccess &&
                            hipEventSynchronize(e1) == hipSuccess &&
                            hipEventElapsedTime(&ms, e0, e1) == hipSuccess && ms > 0.0f;
            (void)hipGetLastError();
            t.release();
            if (!ok) continue;
            const double rate = cellsteps / (ms * 1e-3) / 1e9;
            char line[192];
            snprintf(line, sizeof line, "%s %s %.2f\n", class_name(C).c_str(),
                     cfg_string(C, cand).c_str(), rate);
            report += line;
            if (rate > best_rate) {
                best_rate = rate;
                best = cand;
            }
        }
        C.cfg = best;
        if (best_rate > 0.0) {
            C.tuned_by = "autotune";
            C.gcells = best_rate;
            tune_cache_put(cache_key(C, b->device), cfg_string(C, best), best_rate);
        } else {
            C.cfg = saved;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (hipStreamSynchronize(st) != hipSuccess) return bfail(STENCIL_EDEVICE, "device error while autotuning");
    return batch_build(b);
}

// stencil_run_batched keeps the batches of its last few distinct calls, so
// that a repeated call replays its graph instead of rebuilding it.
struct OneShotKey {
    int device = 0;
    std::vector<uint64_t> serial;
    std::vector<const float *> ins;
    std::vector<float *> outs;
    std::vector<int64_t> steps;
    bool operator==(const OneShotKey &o) const {
        return device == o.device && serial == o.serial && ins == o.ins && outs == o.outs &&
               steps == o.steps;
    }
};

std::mutex g_oneshot_mu;
std::vector<std::pair<OneShotKey, stencil_batch_s *>> g_oneshot;  // most recent last

}  // namespace

extern "C" {

int stencil_batch_create(stencil_batch_t *batch, int n, const stencil_plan_t *plans,
                         const float *const *ins, float *const *outs, const int64_t *steps,
                         const char *tune) {
    star_clear_error();
    return batch_create(batch, n, plans, ins, outs, steps, tune);
}

int stencil_batch_launch(stencil_batch_t batch, void *stream) {
    star_clear_error();
    if (!batch) return bfail(STENCIL_EINVAL, "batch is NULL");
    const hipStream_t st = (hipStream_t)stream;
    const hipError_t e = batch->use_graph ? hipGraphLaunch(batch->exec, st) : enqueue_all(batch, st);
    if (e != hipSuccess) return bhip(e, "batch launch");
    return STENCIL_OK;
}

int stencil_batch_autotune(stencil_batch_t batch, char *report, size_t report_len, void *stream) {
    star_clear_error();
    if (!batch) return bfail(STENCIL_EINVAL, "batch is NULL");
    std::string r;
    const int rc = batch_autotune(batch, r, (hipStream_t)stream);
    if (report && report_len > 0) {
        const size_t k = std::min(report_len - 1, r.size());
        std::memcpy(report, r.data(), k);
        report[k] = '\0';
    }
    return rc;
}

int stencil_batch_describe(stencil_batch_t batch, char *buf, size_t len) {
    star_clear_error();
    if (!batch) return bfail(STENCIL_EINVAL, "batch is NULL");
    std::string s;
    char line[256];
    snprintf(line, sizeof line,
             "grids=%d classes=%zu chains=%zu own=%zu launches=%zu streams=%zu graph=%d\n",
             batch->n, batch->classes.size(), batch->sched.chains.size(), batch->own.size(),
             batch->sched.launches.size(), batch->side.size(), batch->use_graph ? 1 : 0);
    s += line;
    for (size_t c = 0; c < batch->classes.size(); ++c) {
        const BClass &C = batch->classes[c];
        const int ch = batch->sched.chain_of_class.empty() ? -1 : batch->sched.chain_of_class[c];
        snprintf(line, sizeof line, "%s grids=%zu %s by=%s chain=%d launches=%d stream=%d\n",
                 class_name(C).c_str(), C.grids.size(), cfg_string(C, C.cfg).c_str(),
                 C.tuned_by.c_str(), ch,
                 ch < 0 ? 0 : batch->sched.chain_end[ch] - batch->sched.chain_begin[ch],
                 ch < 0 || batch->stream_of_chain.empty() ? 0 : batch->stream_of_chain[ch]);
        s += line;
    }
    if (buf && len > 0) {
        const size_t k = std::min(len - 1, s.size());
        std::memcpy(buf, s.data(), k);
        buf[k] = '\0';
    }
    return (int)s.size();
}

void stencil_batch_destroy(stencil_batch_t batch) { delete batch; }

int stencil_run_batched(int n, const stencil_plan_t *plans, const float *const *ins,
                        float *const *outs, const int64_t *steps, void *stream) {
    star_clear_error();
    if (n < 0) return bfail(STENCIL_EINVAL, "n must be >= 0");
    if (n == 0) return STENCIL_OK;
    if (!plans || !ins || !outs || !steps) return bfail(STENCIL_EINVAL, "NULL batch array");
    OneShotKey key;
    for (int g = 0; g < n; ++g)
        if (!plans[g]) return bfail(STENCIL_EINVAL, "grid %d: plan is NULL", g);
    if (hipGetDevice(&key.device) != hipSuccess) return bhip(hipGetLastError(), "hipGetDevice");
    for (int g = 0; g < n; ++g) key.serial.push_back(plans[g]->serial);
    key.ins.assign(ins, ins + n);
    key.outs.assign(outs, outs + n);
    key.steps.assign(steps, steps + n);
    std::lock_guard<std::mutex> lk(g_oneshot_mu);
    stencil_batch_s *b = nullptr;
    for (size_t i = 0; i < g_oneshot.size(); ++i) {
        if (g_oneshot[i].first == key) {
            auto hit = g_oneshot[i];
            g_oneshot.erase(g_oneshot.begin() + (long)i);
            g_oneshot.push_back(hit);
            b = hit.second;
            break;
        }
    }
    if (!b) {
        const int rc = batch_create(&b, n, plans, ins, outs, steps, nullptr);
        if (rc != STENCIL_OK) return rc;
        if (g_oneshot.size() >= (size_t)kOneShotCache) {
            delete g_oneshot.front().second;
            g_oneshot.erase(g_oneshot.begin());
        }
        g_oneshot.push_back({key, b});
    }
    return stencil_batch_launch(b, stream);
}

}  // extern "C"
