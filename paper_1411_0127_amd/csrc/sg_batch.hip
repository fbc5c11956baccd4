// Batch runtime of libsg: many lattices of different sizes, temperatures and
// sweep counts advanced together.  Each round advances every lattice that still
// has sweeps to do (one work item per tile and z chunk of every lattice): by two
// sweeps on the two-sweep march (one for an odd last sweep), else by one.
//
// Two forms of a run.  Persistent (the default): all rounds of the run in one
// launch of k_batch_persistent, whose workgroups take (round, item) entries from
// one queue per XCD (items dealt to the XCDs as the per-round launch deals them)
// and start a lattice's round as soon as that lattice's previous round is done, so
// lattices never wait for each other; with rounds_per_graph > 0 the
// launch (and the reset of its counters) is captured once into a hipGraph and
// replayed while the run's shape stays the same.  A run of several rounds over
// more lattice memory than group_bytes is split into launches of groups of
// lattices, one after another, so that a launch streams over one group's memory
// rather than the whole resident set.  Per round: one launch of
// k_fused_batch per round, eagerly or from a captured graph of rounds_per_graph
// rounds (the round number lives in device memory, so the graph needs no new
// arguments).  Lattices join and leave between runs: a serving loop admits and
// retires at those boundaries.
//
// Every site update is the same arithmetic as a sweep of the lattice alone, with
// the same keyed streams, so a lattice's spins after n sweeps do not depend on
// what else was in the batch.
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "sg_internal.h"

struct sg_batch {
    struct Job {
        sg_lattice *lat;
        int64_t left;  // sweeps still to do
        double beta;
    };
    hipStream_t stream = nullptr;
    int max_lat = 0, max_items = 0;
    sg::BatchEntry *d_entries = nullptr;
    uint32_t *d_item_lat = nullptr;
    int64_t *d_round = nullptr;
    // persistent runs: queue counters (one per XCD), error flag, per-lattice
    // counters, round tables (one per queue)
    unsigned long long *d_queue = nullptr;
    uint32_t *d_error = nullptr;
    uint32_t *d_done = nullptr;
    uint64_t *d_cum = nullptr;
    bool persistent = true;
    uint32_t spin_cap = 1u << 22;
    // persistent runs: lattices whose spins and couplings (40 B per site) add up to
    // at most this many bytes share one launch; 0: one launch for all
    size_t group_bytes = (size_t)12 << 30;
    // host tables of the groups of the last grouped run (copied from pageable memory,
    // which the runtime stages before the copy call returns; kept until the next run)
    std::vector<std::vector<sg::BatchEntry>> g_entries;
    std::vector<std::vector<uint32_t>> g_items;
    std::vector<std::vector<uint64_t>> g_cum;
    std::vector<uint64_t> h_cum;
    std::vector<int> order;  // job indices in layout order (persistent: by rounds left, descending)
    std::vector<Job> jobs;
    std::vector<sg_lattice *> finished;
    std::vector<sg::BatchEntry> h_entries;
    std::vector<uint32_t> h_item_lat;
    int nitems = 0;
    size_t lds = 0;
    bool layout_dirty = true;
    // captured graph of G rounds for (nitems, lds)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int graph_rounds = 0, graph_items = -1;
    size_t graph_lds = 0;
    bool graph_persistent = false;
    uint64_t graph_total = 0;  // persistent graph: queue entries and lattices it was captured for
    int graph_lat = 0;
};

namespace sg {
namespace {

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

void drop_graph(sg_batch *b)
{
    if (b->exec)
        (void)hipGraphExecDestroy(b->exec);
    if (b->graph)
        (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
    b->graph_rounds = 0;
    b->graph_items = -1;
    b->graph_total = 0;
}

// Persistent runs of fewer rounds than this stay one launch: each group launch ends
// with a drain of its last round, which a run of a round or two does not win back.
constexpr int64_t kMinGroupRounds = 4;

// Rounds one persistent launch covers at most (size of the device round table).
constexpr int kMaxPersistentRounds = 4096;

// Tile of a lattice inside a batch: its chosen (autotuned) tile or the default of
// its kernel; z chunks of the whole column up to L = 512 and half of it above for
// the two-sweep march, of up to 128 planes for the one-sweep march.  Lattices on
// any kernel but SG_KERNEL_FUSED get two-sweep rounds when the tile allows them
// (a batch has no two-pass form: a lattice set to it takes the default march).
int batch_tile(const sg_lattice *lat, BatchEntry &e)
{
    const bool want_two = lat->kernel != SG_KERNEL_FUSED;
    int tx = 0, ty = 0, zc = 0;
    if ((lat->kernel == SG_KERNEL_FUSED || lat->kernel == SG_KERNEL_FUSED2) && lat->tile_x > 0) {
        tx = lat->tile_x;
        ty = lat->tile_y;
    } else if (want_two && lat->L >= 8) {
        fused2_default_shape(lat->L, tx, ty, zc);
    } else {
        fused_default_shape(lat->L, 1, tx, ty, zc);
    }
    // a chunk of the two-sweep march recomputes six planes, of the one-sweep march two
    if (want_two && lat->L >= 8 && fused2_shape_ok(lat->L, tx, ty, 0))
        zc = lat->L <= 512 ? lat->L : lat->L / 2;
    else
        zc = lat->L <= 128 ? lat->L : std::max(64, std::min(128, lat->L / 4));
    if (!fill_batch_entry(e, lat->L, tx, ty, zc, lat->band > 0 ? lat->band : 1, want_two))
        return fail(SG_EINVAL, "no fused tile fits a lattice of side " + std::to_string(lat->L));
    return SG_OK;
}

// Rounds a lattice needs for `left` sweeps.
int64_t rounds_for(const BatchEntry &e, int64_t left) { return e.two ? (left + 1) / 2 : left; }

// Round tables of a persistent launch, one per queue: cum[q * (R + 1) + r] = entries of
// queue q before round r.  Round r has the items of the lattices still active in it,
// which `order` (indices into ent, by rounds needed, most first) puts first, dealt to
// the queues in groups of kBatchGroup, group g to queue g mod kBatchQueues.  Returns
// the entries of all queues.
uint64_t round_tables(const std::vector<BatchEntry> &ent, const std::vector<int> &order, int64_t nitems, int64_t R,
                      std::vector<uint64_t> &cum)
{
    const size_t stride = (size_t)R + 1;
    cum.assign((size_t)kBatchQueues * stride, 0);
    size_t act = order.size();
    int64_t items_act = nitems;
    for (int64_t r = 0; r < R; ++r) {
        while (act > 0) {
            const BatchEntry &en = ent[(size_t)order[act - 1]];
            if (rounds_for(en, en.nsweeps) > r)
                break;
            items_act -= en.nitems;
            --act;
        }
        for (int q = 0; q < kBatchQueues; ++q) {
            int64_t cnt = 0;
            for (int64_t g = q; g * kBatchGroup < items_act; g += kBatchQueues)
                cnt += std::min<int64_t>(kBatchGroup, items_act - g * kBatchGroup);
            cum[(size_t)q * stride + (size_t)r + 1] = cum[(size_t)q * stride + (size_t)r] + (uint64_t)cnt;
        }
    }
    uint64_t total = 0;
    for (int q = 0; q < kBatchQueues; ++q)
        total += cum[(size_t)q * stride + (size_t)R];
    return total;
}

// Lay out the work items of the current jobs (after jobs joined or left).
int build_layout(sg_batch *b)
{
    b->h_entries.assign(b->jobs.size(), BatchEntry{});
    b->h_item_lat.clear();
    size_t lds = 0;
    int items = 0;
    if (b->order.size() != b->jobs.size()) {
        b->order.resize(b->jobs.size());
        for (size_t j = 0; j < b->jobs.size(); ++j)
            b->order[j] = (int)j;
    }
    for (size_t o = 0; o < b->order.size(); ++o) {
        const size_t j = (size_t)b->order[o];
        BatchEntry &e = b->h_entries[j];
        const int rc = batch_tile(b->jobs[j].lat, e);
        if (rc != SG_OK)
            return rc;
        e.item0 = items;
        if ((int64_t)items + e.nitems > b->max_items)
            return fail(SG_EINVAL, "batch work items exceed max_items");
        items += e.nitems;
        b->h_item_lat.insert(b->h_item_lat.end(), (size_t)e.nitems, (uint32_t)j);
        lds = std::max(lds, fused_batch_lds_bytes(e));
    }
    b->nitems = items;
    b->lds = lds;
    b->layout_dirty = false;
    return SG_OK;
}

int record_round(sg_batch *b)
{
    hipError_t e = launch_fused_batch(b->d_entries, b->d_item_lat, b->nitems, b->d_round, b->lds, b->stream);
    if (e == hipSuccess)
        e = launch_round_advance(b->d_round, b->stream);
    return e == hipSuccess ? SG_OK : hip_fail(e, "batch round");
}

}  // namespace
}  // namespace sg

using namespace sg;

extern "C" {

int sg_batch_footprint(int max_lattices, int max_items, size_t *dev_bytes)
{
    if (max_lattices < 1 || max_items < 1 || !dev_bytes)
        return fail(SG_EINVAL, "bad batch size");
    *dev_bytes = align256(sizeof(BatchEntry) * (size_t)max_lattices) + align256(4 * (size_t)max_items) + 256 +
                 align256(4 * (size_t)max_lattices) +
                 align256(8 * (size_t)kBatchQueues * (size_t)(kMaxPersistentRounds + 1)) + 256;
    return SG_OK;
}

int sg_batch_create(int max_lattices, int max_items, void *dev_buf, size_t dev_bytes, void *stream, sg_batch **out)
{
    if (!out)
        return fail(SG_EINVAL, "out is NULL");
    *out = nullptr;
    size_t need = 0;
    if (sg_batch_footprint(max_lattices, max_items, &need) != SG_OK)
        return SG_EINVAL;
    if (!dev_buf || dev_bytes < need)
        return fail(SG_EINVAL, "batch device buffer too small: need " + std::to_string(need) + " bytes");
    if ((reinterpret_cast<uintptr_t>(dev_buf) & 255) != 0)
        return fail(SG_EINVAL, "batch device buffer must be 256-byte aligned");
    sg_batch *b = new (std::nothrow) sg_batch();
    if (!b)
        return fail(SG_ENOMEM, "out of host memory");
    uint8_t *p = static_cast<uint8_t *>(dev_buf);
    b->stream = static_cast<hipStream_t>(stream);
    b->max_lat = max_lattices;
    b->max_items = max_items;
    b->d_entries = reinterpret_cast<BatchEntry *>(p);
    p += align256(sizeof(BatchEntry) * (size_t)max_lattices);
    b->d_item_lat = reinterpret_cast<uint32_t *>(p);
    p += align256(4 * (size_t)max_items);
    static_assert(8 * kBatchQueues <= 64, "queue counters fit between the round counter and the error flag");
    b->d_round = reinterpret_cast<int64_t *>(p);
    b->d_queue = reinterpret_cast<unsigned long long *>(p + 64);
    b->d_error = reinterpret_cast<uint32_t *>(p + 128);
    p += 256;
    b->d_done = reinterpret_cast<uint32_t *>(p);
    p += align256(4 * (size_t)max_lattices);
    b->d_cum = reinterpret_cast<uint64_t *>(p);
    // the error flag is read after runs of either form, so it starts cleared (the
    // caller's buffer holds anything); persistent launches clear it again
    const hipError_t e = launch_batch_reset(b->d_queue, b->d_error, b->d_done, max_lattices, b->stream);
    if (e != hipSuccess) {
        delete b;
        return hip_fail(e, "batch counters");
    }
    *out = b;
    return SG_OK;
}

int sg_batch_add(sg_batch *b, sg_lattice *lat, int64_t nsweeps, double beta)
{
    if (!b || !lat)
        return fail(SG_EINVAL, "NULL argument");
    if (nsweeps < 1)
        return fail(SG_EINVAL, "nsweeps must be >= 1");
    if (std::isnan(beta) || beta < 0)
        return fail(SG_EINVAL, "beta must be >= 0");
    if (lat->prng != SG_MINSTD)
        return fail(SG_EINVAL, "batched sweeps take MINSTD lattices");
    if (lat->stream != b->stream)
        return fail(SG_EMISMATCH, "a batched lattice must use the batch's stream");
    if ((int)b->jobs.size() >= b->max_lat)
        return fail(SG_EINVAL, "batch is full (max_lattices)");
    for (const auto &j : b->jobs)
        if (j.lat == lat)
            return fail(SG_EINVAL, "lattice already in the batch");
    b->jobs.push_back({lat, nsweeps, beta});
    b->layout_dirty = true;
    return SG_OK;
}

int sg_batch_run(sg_batch *b, int64_t max_rounds, int rounds_per_graph, int64_t *rounds_done)
{
    if (!b)
        return fail(SG_EINVAL, "NULL batch");
    if (rounds_done)
        *rounds_done = 0;
    if (max_rounds < 0 || rounds_per_graph < 0)
        return fail(SG_EINVAL, "negative round count");
    if (b->jobs.empty() || max_rounds == 0)
        return SG_OK;
    int rc = SG_OK;
    if (b->persistent) {
        // lattices in order of the rounds they still need, most first: the ones
        // active in a round are then a prefix of the layout
        std::vector<int64_t> need(b->jobs.size());
        for (size_t j = 0; j < b->jobs.size(); ++j) {
            BatchEntry e{};
            rc = batch_tile(b->jobs[j].lat, e);
            if (rc != SG_OK)
                return rc;
            need[j] = rounds_for(e, b->jobs[j].left);
        }
        std::vector<int> order(b->jobs.size());
        for (size_t j = 0; j < order.size(); ++j)
            order[j] = (int)j;
        std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return need[x] > need[y]; });
        if (order != b->order) {
            b->order = order;
            b->layout_dirty = true;
        }
    }
    if (b->layout_dirty) {
        rc = build_layout(b);
        if (rc != SG_OK)
            return rc;
    }
    int64_t R = 0;
    for (size_t j = 0; j < b->jobs.size(); ++j)
        R = std::max(R, rounds_for(b->h_entries[j], b->jobs[j].left));
    R = std::min(R, max_rounds);
    if (b->persistent)
        R = std::min<int64_t>(R, kMaxPersistentRounds);
    // per-run lattice state: sweep count, current buffer, sweeps in this run
    for (size_t j = 0; j < b->jobs.size(); ++j) {
        BatchEntry &e = b->h_entries[j];
        const sg_batch::Job &job = b->jobs[j];
        e.J = job.lat->J;
        e.spins[0] = job.lat->spins[0];
        e.spins[1] = job.lat->spins[1];
        e.mk = job.lat->minstd_k;
        e.c0 = job.lat->cur;
        e.t0 = job.lat->t;
        e.nsweeps = std::min(job.left, e.two ? 2 * R : R);
        uint64_t T[3];
        sg_thresholds(job.beta, SG_MINSTD, T);
        e.t4 = T[0];
        e.t8 = T[1];
        e.t12 = T[2];
    }
    // pageable sources: the runtime stages them before these calls return, so the
    // host vectors may change for the next run right away
    hipError_t e = hipMemcpyAsync(b->d_entries, b->h_entries.data(), sizeof(BatchEntry) * b->h_entries.size(),
                                  hipMemcpyHostToDevice, b->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_item_lat, b->h_item_lat.data(), 4 * b->h_item_lat.size(), hipMemcpyHostToDevice,
                           b->stream);
    if (e == hipSuccess && !b->persistent)
        e = launch_round_reset(b->d_round, b->stream);
    if (e != hipSuccess)
        return hip_fail(e, "batch setup");

    int64_t done = 0;
    const int G = rounds_per_graph;
    // persistent runs: groups of consecutive lattices of the layout order (a group's
    // own order is then by rounds needed too) whose swept bytes stay within
    // group_bytes, one launch each; a launch then streams over one group's memory,
    // not the whole resident set
    std::vector<size_t> gstart{0};
    if (b->persistent && b->group_bytes > 0 && R >= kMinGroupRounds) {
        size_t acc = 0;
        for (size_t o = 0; o < b->order.size(); ++o) {
            const size_t bytes = 40 * (size_t)b->jobs[(size_t)b->order[o]].lat->V;
            if (o > gstart.back() && acc + bytes > b->group_bytes) {
                gstart.push_back(o);
                acc = 0;
            }
            acc += bytes;
        }
    }
    gstart.push_back(b->order.size());
    if (b->persistent && gstart.size() > 2) {
        // launches of the groups one after another on the batch's stream: each one's
        // entries, item table and round tables are copied over the previous ones
        // after that launch (stream order)
        std::vector<std::vector<BatchEntry>> &gent = b->g_entries;
        std::vector<std::vector<uint32_t>> &gitem = b->g_items;
        std::vector<std::vector<uint64_t>> &gcum = b->g_cum;
        gent.assign(gstart.size() - 1, {});
        gitem.assign(gstart.size() - 1, {});
        gcum.assign(gstart.size() - 1, {});
        for (size_t g = 0; g + 1 < gstart.size(); ++g) {
            std::vector<int> gorder;
            int64_t Rg = 0;
            int items = 0;
            for (size_t o = gstart[g]; o < gstart[g + 1]; ++o) {
                BatchEntry en = b->h_entries[(size_t)b->order[o]];
                en.item0 = items;
                gitem[g].insert(gitem[g].end(), (size_t)en.nitems, (uint32_t)(o - gstart[g]));
                items += en.nitems;
                Rg = std::max(Rg, rounds_for(en, en.nsweeps));
                gorder.push_back((int)(o - gstart[g]));
                gent[g].push_back(en);
            }
            if (Rg == 0)
                continue;
            const uint64_t total = round_tables(gent[g], gorder, items, Rg, gcum[g]);
            e = hipMemcpyAsync(b->d_entries, gent[g].data(), sizeof(BatchEntry) * gent[g].size(),
                               hipMemcpyHostToDevice, b->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(b->d_item_lat, gitem[g].data(), 4 * gitem[g].size(), hipMemcpyHostToDevice,
                                   b->stream);
            if (e == hipSuccess)
                e = hipMemcpyAsync(b->d_cum, gcum[g].data(), 8 * gcum[g].size(), hipMemcpyHostToDevice, b->stream);
            if (e == hipSuccess)
                e = launch_batch_persistent(b->d_entries, b->d_item_lat, b->d_cum, (int)Rg, b->d_queue, b->d_done,
                                            b->d_error, (int)gent[g].size(), b->spin_cap, b->lds, (int64_t)total,
                                            b->stream);
            if (e != hipSuccess)
                return hip_fail(e, "grouped persistent batch launch");
        }
        done = R;
    } else if (b->persistent) {
        uint64_t total = round_tables(b->h_entries, b->order, b->nitems, R, b->h_cum);
        e = hipMemcpyAsync(b->d_cum, b->h_cum.data(), 8 * b->h_cum.size(), hipMemcpyHostToDevice, b->stream);
        if (e != hipSuccess)
            return hip_fail(e, "batch round table");
        auto record = [&]() -> hipError_t {
            return launch_batch_persistent(b->d_entries, b->d_item_lat, b->d_cum, (int)R, b->d_queue, b->d_done,
                                           b->d_error, (int)b->jobs.size(), b->spin_cap, b->lds, (int64_t)total,
                                           b->stream);
        };
        if (G > 0) {
            // the launch reads everything that changes between runs from device
            // memory, so one captured graph serves every run of the same shape
            if (!b->exec || !b->graph_persistent || b->graph_rounds != (int)R || b->graph_total != total ||
                b->graph_lds != b->lds || b->graph_items != b->nitems || b->graph_lat != (int)b->jobs.size()) {
                drop_graph(b);
                e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
                if (e != hipSuccess)
                    return hip_fail(e, "begin capture");
                const hipError_t le = record();
                hipGraph_t graph = nullptr;
                e = hipStreamEndCapture(b->stream, &graph);
                if (le != hipSuccess) {
                    if (graph)
                        (void)hipGraphDestroy(graph);
                    return hip_fail(le, "persistent batch launch");
                }
                if (e != hipSuccess)
                    return hip_fail(e, "end capture");
                b->graph = graph;
                e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
                if (e != hipSuccess) {
                    drop_graph(b);
                    return hip_fail(e, "graph instantiate");
                }
                b->graph_persistent = true;
                b->graph_rounds = (int)R;
                b->graph_total = total;
                b->graph_lat = (int)b->jobs.size();
                b->graph_lds = b->lds;
                b->graph_items = b->nitems;
            }
            e = hipGraphLaunch(b->exec, b->stream);
        } else {
            e = record();
        }
        if (e != hipSuccess)
            return hip_fail(e, "persistent batch launch");
        done = R;
    } else if (G > 0 && R >= G) {
        if (!b->exec || b->graph_persistent || b->graph_rounds != G || b->graph_items != b->nitems ||
            b->graph_lds != b->lds) {
            drop_graph(b);
            e = hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal);
            if (e != hipSuccess)
                return hip_fail(e, "begin capture");
            for (int g = 0; g < G && rc == SG_OK; ++g)
                rc = record_round(b);
            hipGraph_t graph = nullptr;
            e = hipStreamEndCapture(b->stream, &graph);
            if (rc != SG_OK) {
                if (graph)
                    (void)hipGraphDestroy(graph);
                return rc;
            }
            if (e != hipSuccess)
                return hip_fail(e, "end capture");
            b->graph = graph;
            e = hipGraphInstantiate(&b->exec, graph, nullptr, nullptr, 0);
            if (e != hipSuccess) {
                drop_graph(b);
                return hip_fail(e, "graph instantiate");
            }
            b->graph_persistent = false;
            b->graph_rounds = G;
            b->graph_items = b->nitems;
            b->graph_lds = b->lds;
        }
        for (; done + G <= R; done += G) {
            e = hipGraphLaunch(b->exec, b->stream);
            if (e != hipSuccess)
                return hip_fail(e, "graph launch");
        }
    }
    for (; done < R; ++done) {
        rc = record_round(b);
        if (rc != SG_OK)
            return rc;
    }
    // the host view of every lattice moves with the queued rounds
    std::vector<sg_batch::Job> keep;
    for (size_t j = 0; j < b->jobs.size(); ++j) {
        sg_batch::Job &job = b->jobs[j];
        const BatchEntry &en = b->h_entries[j];
        const int64_t d = en.nsweeps;  // sweeps done in this run
        job.lat->t += d;
        job.lat->cur ^= (int)(rounds_for(en, d) & 1);
        job.left -= d;
        if (job.left == 0)
            b->finished.push_back(job.lat);
        else
            keep.push_back(job);
    }
    if (keep.size() != b->jobs.size()) {
        b->layout_dirty = true;
        b->order.clear();
    }
    b->jobs.swap(keep);
    if (rounds_done)
        *rounds_done = done;
    return SG_OK;
}

int sg_batch_set_persistent(sg_batch *b, int on, uint32_t spin_cap)
{
    if (!b)
        return fail(SG_EINVAL, "NULL batch");
    if (on != 0 && on != 1)
        return fail(SG_EINVAL, "on must be 0 or 1");
    if ((on != 0) != b->persistent)
        drop_graph(b);
    b->persistent = on != 0;
    b->spin_cap = spin_cap == 0 ? (1u << 22) : spin_cap;
    return SG_OK;
}

int sg_batch_set_group_bytes(sg_batch *b, size_t bytes)
{
    if (!b)
        return fail(SG_EINVAL, "NULL batch");
    b->group_bytes = bytes;
    return SG_OK;
}

int sg_batch_check(sg_batch *b)
{
    if (!b)
        return fail(SG_EINVAL, "NULL batch");
    uint32_t err = 0;
    hipError_t e = hipMemcpyAsync(&err, b->d_error, 4, hipMemcpyDeviceToHost, b->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(b->stream);
    if (e != hipSuccess)
        return hip_fail(e, "batch check");
    if (err != 0)
        return fail(SG_EDEVICE, "a persistent batch run gave up waiting for a round (spin limit reached); the "
                                "lattices of that run are not valid");
    return SG_OK;
}

int sg_batch_take_finished(sg_batch *b, sg_lattice **out, int max, int *n)
{
    if (!b || !n || (max > 0 && !out))
        return fail(SG_EINVAL, "NULL argument");
    int k = 0;
    while (k < max && !b->finished.empty()) {
        out[k++] = b->finished.front();
        b->finished.erase(b->finished.begin());
    }
    *n = k;
    return SG_OK;
}

int sg_batch_size(const sg_batch *b, int *active, int *finished, int *items)
{
    if (!b)
        return fail(SG_EINVAL, "NULL batch");
    if (active)
        *active = (int)b->jobs.size();
    if (finished)
        *finished = (int)b->finished.size();
    if (items) {
        int n = 0;
        for (const auto &job : b->jobs) {
            BatchEntry e{};
            if (batch_tile(job.lat, e) == SG_OK)
                n += e.nitems;
        }
        *items = n;
    }
    return SG_OK;
}

int sg_batch_rounds_left(const sg_batch *b, int64_t *first, int64_t *last)
{
    if (!b)
        return fail(SG_EINVAL, "NULL batch");
    int64_t lo = 0, hi = 0;
    bool any = false;
    for (const auto &job : b->jobs) {
        BatchEntry e{};
        const int rc = batch_tile(job.lat, e);
        if (rc != SG_OK)
            return rc;
        const int64_t n = rounds_for(e, job.left);
        lo = any ? std::min(lo, n) : n;
        hi = any ? std::max(hi, n) : n;
        any = true;
    }
    if (first)
        *first = lo;
    if (last)
        *last = hi;
    return SG_OK;
}

int sg_batch_destroy(sg_batch *b)
{
    if (!b)
        return SG_OK;
    drop_graph(b);
    delete b;
    return SG_OK;
}

}  // extern "C"
