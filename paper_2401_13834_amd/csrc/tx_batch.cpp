// Batches: the jobs of many beams (uneven channel counts, block lengths and DM
// grids, each with its own plan's tile variants) run as persistent launches:
// one per first-stage variant, one per (second-stage trials per workgroup,
// variant) class and one for the boxcar of every job, each a grid of what the
// device holds at once whose workgroups take tile after tile from work
// counters in device memory.  Optionally the launches are captured in a HIP
// graph.  The job tables and counters live in device memory and are uploaded
// before every launch, so a captured graph can be replayed over a different
// set of jobs.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "tx_internal.h"

namespace {

constexpr int kIWs[] = {16, 13, 8, 4, 2, 1};
constexpr int kNIW = 6;
constexpr int kQueues = 8;           // work counters per launch (one per XCD's eighth of the items)

int iw_index(int iw) {
    for (int k = 0; k < kNIW; ++k)
        if (kIWs[k] == iw) return k;
    return -1;
}

int n_s1() { return tx::stage1_variant_count(); }
int n_s2() { return kNIW * tx::stage2_variant_count(); }   // classes (iw, variant)
int s2_class(int iw, int variant) { return iw_index(iw) * tx::stage2_variant_count() + variant; }

struct Job {
    tx_plan_s* plan = nullptr;
    tx_stream_s* stream = nullptr;     // stream job: input is the stream's history + block
    const uint8_t* in = nullptr;       // device block, or the block pushed to the stream
    int64_t in_pitch = 0;
    int64_t nt = 0;                    // output samples (device job) / pushed samples (stream job)
    int block_on_device = 1;
    bool time_major = false;           // stream job: the block is [nt][nchan] (transposed on ingest)
    int32_t* out = nullptr;
    int64_t out_pitch = 0;
    bool has_box = false;
    tx::BoxcarArgs box{};
    int64_t nt_out = 0;                // outputs produced by the last launch
};

// Layout of the integer table, for max_jobs M: per launch class its info
// (jobs, first job, first prefix entry), the tile prefix sums of each stage
// (a class's segment holds its jobs + 1 entries) and the work counters.
struct IntLayout {
    int M = 0, C1 = 0, C2 = 0;
    int info1(int c) const { return 3 * c; }
    int info2(int c) const { return 3 * (C1 + c); }
    int infob() const { return 3 * (C1 + C2); }
    int pre1() const { return infob() + 3; }
    int pre2() const { return pre1() + M + C1; }
    int preb() const { return pre2() + M + C2; }
    int q1(int c) const { return preb() + M + 1 + kQueues * c; }
    int q2(int c) const { return q1(C1) + kQueues * c; }
    int qb() const { return q2(C2); }
    int size() const { return qb() + kQueues; }
};

struct Signature {            // what a captured graph bakes in
    std::vector<int> lds1;    // per first-stage class: dynamic LDS (0 = not launched)
    std::vector<int> lds2;    // per second-stage class
    int nwt = 0;              // boxcar instance (0 = no boxcar)
    int ldsb = 0;             // boxcar dynamic LDS (per-(tile, width) maxima)
    void init() {
        lds1.assign(static_cast<size_t>(n_s1()), 0);
        lds2.assign(static_cast<size_t>(n_s2()), 0);
        nwt = 0;
        ldsb = 0;
    }
    void merge(const Signature& o) {
        for (size_t c = 0; c < lds1.size(); ++c) lds1[c] = std::max(lds1[c], o.lds1[c]);
        for (size_t c = 0; c < lds2.size(); ++c) lds2[c] = std::max(lds2[c], o.lds2[c]);
        nwt = std::max(nwt, o.nwt);
        ldsb = std::max(ldsb, o.ldsb);
    }
    // Every kernel of `need` is in this signature with at least its LDS.
    bool holds(const Signature& need) const {
        for (size_t c = 0; c < lds1.size(); ++c)
            if (need.lds1[c] > 0 && lds1[c] < need.lds1[c]) return false;
        for (size_t c = 0; c < lds2.size(); ++c)
            if (need.lds2[c] > 0 && lds2[c] < need.lds2[c]) return false;
        return need.nwt == 0 || nwt >= need.nwt;
    }
};

}  // namespace

struct tx_batch_s {
    int device = -1;
    int max_jobs = 0;
    uint32_t flags = 0;
    std::vector<Job> jobs;
    IntLayout L;
    // device tables and their pinned host mirror (one contiguous block)
    size_t off_s1 = 0, off_s2 = 0, off_bx = 0, off_int = 0, table_bytes = 0;
    uint8_t* d_tab = nullptr;
    uint8_t* h_tab = nullptr;
    hipEvent_t uploaded = nullptr;     // the last upload from h_tab has been consumed
    bool upload_pending = false;
    hipEvent_t finished = nullptr;     // recorded after the last launch's work
    bool launched = false;
    // first-stage series of every job of a launch
    void* scratch = nullptr;
    int64_t scratch_bytes = 0;
    // the captured graph (TX_BATCH_GRAPH) and the kernels it holds
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    Signature captured;
    // plans declared ahead of the first launch (tx_batch_reserve): the union
    // of their kernels and LDS sizes
    bool reserved = false;
    Signature floor;
};

namespace {

void destroy_graph(tx_batch_s* b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->exec = nullptr;
    b->graph = nullptr;
}

tx_status fill_box(const tx_batch_boxcar* box, tx::BoxcarArgs* a) {
    *a = tx::BoxcarArgs{};
    if (!box->d_snr || !box->d_width || !box->d_time) return TX_EINVAL;
    tx_status st = tx::boxcar_widths(box->widths, box->nw, TX_MAX_NT_BOXCAR, a);
    if (st != TX_OK) return st;
    const bool cands = box->d_cands || box->d_count;
    if (cands && (!box->d_count || box->cap < 0 || (box->cap > 0 && !box->d_cands) || !std::isfinite(box->gamma)))
        return TX_EINVAL;
    a->gamma = box->gamma;
    a->want_peaks = 1;
    a->want_cands = cands ? 1 : 0;
    a->snr = box->d_snr;
    a->width = box->d_width;
    a->time = box->d_time;
    a->cands = box->d_cands;
    a->cap = box->cap;
    a->count = reinterpret_cast<unsigned long long*>(box->d_count);
    return TX_OK;
}

// Kernels a job of `plan` with `nt` outputs (nw boxcar widths, 0 for none)
// needs: its first- and second-stage classes and their LDS, its boxcar.
tx_status job_needs(const tx_plan_s* plan, int64_t nt, int nw, Signature* need, tx::DedispGeom* geo_out) {
    const tx::DedispGeom g = tx::dedisp_geometry(plan, std::max<int64_t>(nt, 1), tx::plan_tiles(plan));
    if (!g.ok) return TX_ENOTSUP;
    need->lds1[static_cast<size_t>(g.tiles.s1)] = std::max(need->lds1[static_cast<size_t>(g.tiles.s1)], g.lds1);
    const int c2 = s2_class(g.iw, g.tiles.s2);
    need->lds2[static_cast<size_t>(c2)] = std::max(need->lds2[static_cast<size_t>(c2)], g.lds2);
    if (nw > 0) {
        need->nwt = std::max(need->nwt, tx::boxcar_nwt(nw));
        need->ldsb = std::max(need->ldsb, tx::boxcar_tmax_bytes(need->nwt, nt));
    }
    if (geo_out) *geo_out = g;
    return TX_OK;
}

// Kernel launches of one batch launch (captured or direct).  tiles*: work
// items per launch class, for direct launches (a graph passes none and gets
// grids that hold any number).
hipError_t run_kernels(tx_batch_s* b, const Signature& sig, hipStream_t st, const std::vector<int64_t>* t1,
                       const std::vector<int64_t>* t2, int64_t tb) {
    int* ints = reinterpret_cast<int*>(b->d_tab + b->off_int);
    const auto* s1 = reinterpret_cast<const tx::Stage1Args*>(b->d_tab + b->off_s1);
    const auto* s2 = reinterpret_cast<const tx::Stage2Args*>(b->d_tab + b->off_s2);
    const auto* bx = reinterpret_cast<const tx::BoxcarArgs*>(b->d_tab + b->off_bx);
    uint32_t* q = reinterpret_cast<uint32_t*>(ints);
    const IntLayout& L = b->L;
    hipError_t e = hipSuccess;
    if (sig.nwt > 0) {
        e = tx::launch_zero_counts(bx, ints + L.infob(), b->max_jobs, st);
        if (e != hipSuccess) return e;
    }
    for (int c = 0; c < L.C1; ++c) {
        if (sig.lds1[static_cast<size_t>(c)] <= 0) continue;
        const int64_t tiles = t1 ? (*t1)[static_cast<size_t>(c)] : 0;
        if (t1 && tiles == 0) continue;
        const tx::BatchRefs r{s1, ints + L.pre1(), ints + L.info1(c), q + L.q1(c)};
        e = tx::launch_stage1_batch(c, sig.lds1[static_cast<size_t>(c)], r, tiles, st);
        if (e != hipSuccess) return e;
    }
    const int nv2 = tx::stage2_variant_count();
    for (int c = 0; c < L.C2; ++c) {
        if (sig.lds2[static_cast<size_t>(c)] <= 0) continue;
        const int64_t tiles = t2 ? (*t2)[static_cast<size_t>(c)] : 0;
        if (t2 && tiles == 0) continue;
        const tx::BatchRefs r{s2, ints + L.pre2(), ints + L.info2(c), q + L.q2(c)};
        e = tx::launch_stage2_batch(kIWs[c / nv2], c % nv2, sig.lds2[static_cast<size_t>(c)], r, tiles, st);
        if (e != hipSuccess) return e;
    }
    if (sig.nwt > 0 && (!t1 || tb > 0)) {
        const tx::BatchRefs r{bx, ints + L.preb(), ints + L.infob(), q + L.qb()};
        e = tx::launch_boxcar_batch(sig.nwt, sig.ldsb, r, t1 ? tb : 0, st);
    }
    return e;
}

}  // namespace

extern "C" {

tx_status tx_batch_create(int32_t max_jobs, uint32_t flags, tx_batch_t* out) {
    if (!out || max_jobs < 1 || max_jobs > (1 << 20) || (flags & ~TX_BATCH_GRAPH)) return TX_EINVAL;
    *out = nullptr;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return TX_EDEVICE;
    tx_batch_s* b = new (std::nothrow) tx_batch_s();
    if (!b) return TX_ENOMEM;
    b->device = dev;
    b->max_jobs = max_jobs;
    b->flags = flags;
    b->L.M = max_jobs;
    b->L.C1 = n_s1();
    b->L.C2 = n_s2();
    b->captured.init();
    b->floor.init();
    auto align = [](size_t v) { return (v + 255) / 256 * 256; };
    b->off_s1 = 0;
    b->off_s2 = align(sizeof(tx::Stage1Args) * max_jobs);
    b->off_bx = b->off_s2 + align(sizeof(tx::Stage2Args) * max_jobs);
    b->off_int = b->off_bx + align(sizeof(tx::BoxcarArgs) * max_jobs);
    b->table_bytes = b->off_int + align(sizeof(int) * b->L.size());
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&b->d_tab), b->table_bytes);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&b->h_tab), b->table_bytes);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->uploaded, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->finished, hipEventDisableTiming);
    if (e != hipSuccess) {
        tx_batch_destroy(b);
        return tx::status_of(e);
    }
    // Zero, and the work counters stay zero in the mirror: every upload
    // resets them on the device.
    std::memset(b->h_tab, 0, b->table_bytes);
    b->jobs.reserve(static_cast<size_t>(max_jobs));
    *out = b;
    return TX_OK;
}

tx_status tx_batch_clear(tx_batch_t b) {
    if (!b) return TX_EINVAL;
    b->jobs.clear();
    return TX_OK;
}

tx_status tx_batch_add(tx_batch_t b, tx_plan_t plan, const uint8_t* d_in, int64_t in_pitch, int64_t nt,
                       int32_t* d_out, int64_t out_pitch, const tx_batch_boxcar* box) {
    if (!b || !plan) return TX_EINVAL;
    if (static_cast<int>(b->jobs.size()) >= b->max_jobs) return TX_EINVAL;
    if (!plan->on_device || plan->device != b->device) return TX_ESTATE;
    if (nt < 1 || nt > (int64_t(1) << 30) || !d_in || (reinterpret_cast<uintptr_t>(d_in) & 15) || (in_pitch & 15) ||
        in_pitch < nt + plan->overlap)
        return TX_EINVAL;
    tx_status st = tx::check_out_args(d_out, out_pitch, nt);
    if (st != TX_OK) return st;
    Job j;
    j.plan = plan;
    j.in = d_in;
    j.in_pitch = in_pitch;
    j.nt = nt;
    j.out = d_out;
    j.out_pitch = out_pitch;
    if (box) {
        if (nt > TX_MAX_NT_BOXCAR) return TX_EINVAL;
        st = fill_box(box, &j.box);
        if (st != TX_OK) return st;
        j.has_box = true;
    }
    b->jobs.push_back(j);
    return TX_OK;
}

static tx_status add_stream_job(tx_batch_t b, tx_stream_t s, const uint8_t* block, int64_t block_pitch, int64_t nt,
                                int32_t block_on_device, bool time_major, int32_t* d_out, int64_t out_pitch,
                                const tx_batch_boxcar* box) {
    if (!b || !s || !block) return TX_EINVAL;
    if (static_cast<int>(b->jobs.size()) >= b->max_jobs) return TX_EINVAL;
    if (s->device != b->device) return TX_ESTATE;
    for (const Job& o : b->jobs)
        if (o.stream == s) return TX_EINVAL;
    if (nt < 1 || nt > s->max_block || block_pitch < (time_major ? s->plan->nchan : nt)) return TX_EINVAL;
    if (time_major && block_on_device && ((reinterpret_cast<uintptr_t>(block) & 15) || (block_pitch & 15)))
        return TX_EINVAL;
    tx_status st = tx::check_out_args(d_out, out_pitch, nt);
    if (st != TX_OK) return st;
    Job j;
    j.plan = s->plan;
    j.stream = s;
    j.in = block;
    j.in_pitch = block_pitch;
    j.nt = nt;
    j.block_on_device = block_on_device ? 1 : 0;
    j.time_major = time_major;
    j.out = d_out;
    j.out_pitch = out_pitch;
    if (box) {
        if (nt > TX_MAX_NT_BOXCAR) return TX_EINVAL;
        st = fill_box(box, &j.box);
        if (st != TX_OK) return st;
        j.has_box = true;
    }
    b->jobs.push_back(j);
    return TX_OK;
}

tx_status tx_batch_add_stream(tx_batch_t b, tx_stream_t s, const uint8_t* block, int64_t block_pitch, int64_t nt,
                              int32_t block_on_device, int32_t* d_out, int64_t out_pitch,
                              const tx_batch_boxcar* box) {
    return add_stream_job(b, s, block, block_pitch, nt, block_on_device, false, d_out, out_pitch, box);
}

tx_status tx_batch_add_stream_tf(tx_batch_t b, tx_stream_t s, const uint8_t* block, int64_t block_pitch,
                                 int64_t nt, int32_t block_on_device, int32_t* d_out, int64_t out_pitch,
                                 const tx_batch_boxcar* box) {
    return add_stream_job(b, s, block, block_pitch, nt, block_on_device, true, d_out, out_pitch, box);
}

tx_status tx_batch_reserve(tx_batch_t b, tx_plan_t plan, int32_t nw, int64_t max_nt, int32_t count) {
    if (!b || !plan || nw < 0 || nw > TX_MAX_WIDTHS || max_nt < 1 || max_nt > (int64_t(1) << 30) || count < 1 ||
        count > b->max_jobs)
        return TX_EINVAL;
    if (!plan->on_device || plan->device != b->device) return TX_ESTATE;
    Signature need;
    need.init();
    const tx_status st = job_needs(plan, max_nt, nw, &need, nullptr);
    if (st != TX_OK) return st;
    b->floor.merge(need);
    b->reserved = true;
    return TX_OK;
}

tx_status tx_batch_stream_output(tx_batch_t b, int32_t job, int64_t* nt_out) {
    if (!b || !nt_out || job < 0 || job >= static_cast<int32_t>(b->jobs.size())) return TX_EINVAL;
    *nt_out = b->jobs[job].nt_out;
    return TX_OK;
}

tx_status tx_batch_launch(tx_batch_t b, hipStream_t stream) {
    if (!b || b->jobs.empty()) return TX_EINVAL;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return TX_EDEVICE;
    if (dev != b->device) return TX_ESTATE;
    const int n = static_cast<int>(b->jobs.size());
    const bool use_graph = (b->flags & TX_BATCH_GRAPH) && stream != nullptr;

    // Kernels and LDS this launch needs (each job with its plan's own tiles;
    // a graph about to be captured also covers stream jobs at their largest
    // block and the reserved plans).
    Signature need;
    need.init();
    for (const Job& j : b->jobs) {
        const int64_t nt_cap = j.stream ? j.stream->max_block : j.nt;
        const tx_status st = job_needs(j.plan, nt_cap, j.has_box ? j.box.nw : 0, &need, nullptr);
        if (st != TX_OK) return st;
    }
    Signature sig;
    if (use_graph && b->exec) {
        if (!b->captured.holds(need)) return TX_ESTATE;      // before anything is queued
        sig = b->captured;
    } else {
        sig = need;
        if (use_graph) sig.merge(b->floor);
    }

    // Stream jobs: copy each block behind its history (this fixes nt_out).
    for (Job& j : b->jobs) {
        j.nt_out = j.nt;
        if (j.stream) {
            int64_t n_out = 0;
            const tx_status st =
                j.time_major ? tx::stream_ingest_tf(j.stream, j.in, j.in_pitch, j.nt, j.block_on_device, stream, &n_out)
                             : tx::stream_ingest(j.stream, j.in, j.in_pitch, j.nt, j.block_on_device, stream, &n_out);
            if (st != TX_OK) return st;
            j.nt_out = n_out;
        }
    }
    std::vector<tx::DedispGeom> geo(static_cast<size_t>(n));
    std::vector<int64_t> scratch_off(static_cast<size_t>(n), 0);
    int64_t scratch_need = 0;
    for (int k = 0; k < n; ++k) {
        Job& j = b->jobs[static_cast<size_t>(k)];
        geo[static_cast<size_t>(k)] = tx::dedisp_geometry(j.plan, std::max<int64_t>(j.nt_out, 1), tx::plan_tiles(j.plan));
        if (!geo[static_cast<size_t>(k)].ok) return TX_ENOTSUP;
        if (j.nt_out > 0) {
            scratch_off[static_cast<size_t>(k)] = scratch_need;
            scratch_need += geo[static_cast<size_t>(k)].ws_bytes;
        }
    }
    // First-stage scratch of every job (stream-ordered, so in-flight work
    // keeps the old buffer until it is done).
    if (scratch_need > b->scratch_bytes) {
        if (b->scratch) (void)hipFreeAsync(b->scratch, stream);
        b->scratch = nullptr;
        const tx_status rp = tx::retain_pool(b->device);
        if (rp != TX_OK) return rp;
        const hipError_t e = hipMallocAsync(&b->scratch, static_cast<size_t>(scratch_need), stream);
        if (e != hipSuccess) {
            b->scratch_bytes = 0;
            return tx::status_of(e);
        }
        b->scratch_bytes = scratch_need;
    }
    // Job tables into the pinned mirror (after the previous upload was
    // consumed), grouped by launch class.
    if (b->upload_pending) {
        const hipError_t e = hipEventSynchronize(b->uploaded);
        if (e != hipSuccess) return tx::status_of(e);
        b->upload_pending = false;
    }
    const IntLayout& L = b->L;
    auto* h1 = reinterpret_cast<tx::Stage1Args*>(b->h_tab + b->off_s1);
    auto* h2 = reinterpret_cast<tx::Stage2Args*>(b->h_tab + b->off_s2);
    auto* hb = reinterpret_cast<tx::BoxcarArgs*>(b->h_tab + b->off_bx);
    int* hi = reinterpret_cast<int*>(b->h_tab + b->off_int);
    std::vector<int> cls1(static_cast<size_t>(n), -1), cls2(static_cast<size_t>(n), -1);
    std::vector<int> cnt1(static_cast<size_t>(L.C1), 0), cnt2(static_cast<size_t>(L.C2), 0);
    for (int k = 0; k < n; ++k) {
        if (b->jobs[static_cast<size_t>(k)].nt_out <= 0) continue;
        const tx::DedispGeom& g = geo[static_cast<size_t>(k)];
        cls1[static_cast<size_t>(k)] = g.tiles.s1;
        cls2[static_cast<size_t>(k)] = s2_class(g.iw, g.tiles.s2);
        ++cnt1[static_cast<size_t>(g.tiles.s1)];
        ++cnt2[static_cast<size_t>(cls2[static_cast<size_t>(k)])];
    }
    std::vector<int64_t> tiles1(static_cast<size_t>(L.C1), 0), tiles2(static_cast<size_t>(L.C2), 0);
    std::vector<int> fill1(static_cast<size_t>(L.C1), 0), fill2(static_cast<size_t>(L.C2), 0);
    {
        int off = 0;
        for (int c = 0; c < L.C1; ++c) {
            hi[L.info1(c)] = cnt1[static_cast<size_t>(c)];
            hi[L.info1(c) + 1] = off;
            hi[L.info1(c) + 2] = off + c;
            hi[L.pre1() + off + c] = 0;
            fill1[static_cast<size_t>(c)] = off;
            off += cnt1[static_cast<size_t>(c)];
        }
        off = 0;
        for (int c = 0; c < L.C2; ++c) {
            hi[L.info2(c)] = cnt2[static_cast<size_t>(c)];
            hi[L.info2(c) + 1] = off;
            hi[L.info2(c) + 2] = off + c;
            hi[L.pre2() + off + c] = 0;
            fill2[static_cast<size_t>(c)] = off;
            off += cnt2[static_cast<size_t>(c)];
        }
    }
    int nb = 0;
    hi[L.preb()] = 0;
    for (int k = 0; k < n; ++k) {
        Job& j = b->jobs[static_cast<size_t>(k)];
        if (j.nt_out <= 0) continue;
        const tx::DedispGeom& g = geo[static_cast<size_t>(k)];
        tx::Stage1Args a1;
        tx::Stage2Args a2;
        const uint8_t* in = j.in;
        int x_off = 0;
        if (j.stream) tx::stream_input(j.stream, &in, &x_off);
        const int64_t in_pitch = j.stream ? j.stream->pitch : j.in_pitch;
        uint16_t* ws = reinterpret_cast<uint16_t*>(static_cast<uint8_t*>(b->scratch) + scratch_off[static_cast<size_t>(k)]);
        tx::fill_stage_args(j.plan, g, in, in_pitch, j.nt_out, j.out, j.out_pitch, ws, &a1, &a2);
        a1.x_off = x_off;
        const int c1 = cls1[static_cast<size_t>(k)], c2 = cls2[static_cast<size_t>(k)];
        a1.lds_bytes = sig.lds1[static_cast<size_t>(c1)];
        a2.lds_bytes = sig.lds2[static_cast<size_t>(c2)];
        {
            const int pos = fill1[static_cast<size_t>(c1)]++;          // job slot; prefix entry pos + c1 + 1
            h1[pos] = a1;
            hi[L.pre1() + pos + c1 + 1] = hi[L.pre1() + pos + c1] + static_cast<int>(tx::stage1_tiles(a1));
            tiles1[static_cast<size_t>(c1)] += tx::stage1_tiles(a1);
        }
        {
            const int pos = fill2[static_cast<size_t>(c2)]++;
            h2[pos] = a2;
            hi[L.pre2() + pos + c2 + 1] = hi[L.pre2() + pos + c2] + static_cast<int>(tx::stage2_tiles(a2));
            tiles2[static_cast<size_t>(c2)] += tx::stage2_tiles(a2);
        }
        if (j.has_box) {
            tx::BoxcarArgs bx = j.box;
            bx.y = j.out;
            bx.pitch = j.out_pitch;
            bx.ndm = j.plan->ndm;
            bx.nt = static_cast<int32_t>(j.nt_out);
            tx::boxcar_fit(&bx, j.box.widths, j.box.nw, j.nt_out);
            const int need_b = tx::boxcar_tmax_bytes(sig.nwt, j.nt_out);
            bx.tmax_ok = (need_b > 0 && need_b <= sig.ldsb) ? 1 : 0;
            hb[nb] = bx;
            hi[L.preb() + nb + 1] = hi[L.preb() + nb] + bx.ndm;
            ++nb;
        }
    }
    hi[L.infob()] = nb;
    hi[L.infob() + 1] = 0;
    hi[L.infob() + 2] = 0;
    for (int c = 0; c < L.C1; ++c)
        if (tiles1[static_cast<size_t>(c)] > INT32_MAX) return TX_ENOTSUP;
    for (int c = 0; c < L.C2; ++c)
        if (tiles2[static_cast<size_t>(c)] > INT32_MAX) return TX_ENOTSUP;
    hipError_t e = hipMemcpyAsync(b->d_tab, b->h_tab, b->table_bytes, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipEventRecord(b->uploaded, stream);
    if (e != hipSuccess) return tx::status_of(e);
    b->upload_pending = true;

    // Kernels.
    if (use_graph) {
        if (!b->exec) {
            e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                const hipError_t ek = run_kernels(b, sig, stream, nullptr, nullptr, 0);
                hipGraph_t g = nullptr;
                e = hipStreamEndCapture(stream, &g);
                if (ek != hipSuccess) e = ek;
                if (e == hipSuccess) {
                    b->graph = g;
                    e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
                } else if (g) {
                    (void)hipGraphDestroy(g);
                }
            }
            if (e != hipSuccess) {
                destroy_graph(b);
                return tx::status_of(e);
            }
            b->captured = sig;
        }
        e = hipGraphLaunch(b->exec, stream);
    } else {
        int64_t rows = 0;
        for (int k = 0; k < nb; ++k) rows += hb[k].ndm;
        e = run_kernels(b, sig, stream, &tiles1, &tiles2, rows);
    }
    if (e != hipSuccess) return tx::status_of(e);
    // Stream jobs: keep the last `overlap` samples.
    for (Job& j : b->jobs) {
        if (!j.stream) continue;
        const tx_status st = tx::stream_advance(j.stream, j.nt, stream);
        if (st != TX_OK) return st;
    }
    e = hipEventRecord(b->finished, stream);
    if (e != hipSuccess) return tx::status_of(e);
    b->launched = true;
    return TX_OK;
}

tx_status tx_batch_wait(tx_batch_t b) {
    if (!b) return TX_EINVAL;
    if (!b->launched) return TX_OK;
    return tx::status_of(hipEventSynchronize(b->finished));
}

tx_status tx_batch_query(tx_batch_t b, int32_t* done) {
    if (!b || !done) return TX_EINVAL;
    if (!b->launched) {
        *done = 1;
        return TX_OK;
    }
    const hipError_t e = hipEventQuery(b->finished);
    if (e == hipErrorNotReady) {
        (void)hipGetLastError();
        *done = 0;
        return TX_OK;
    }
    *done = e == hipSuccess ? 1 : 0;
    return tx::status_of(e);
}

tx_status tx_batch_destroy(tx_batch_t b) {
    if (!b) return TX_OK;
    if (b->upload_pending) (void)hipEventSynchronize(b->uploaded);
    destroy_graph(b);
    if (b->scratch) {
        (void)hipDeviceSynchronize();
        (void)hipFreeAsync(b->scratch, nullptr);
        (void)hipStreamSynchronize(nullptr);
    }
    if (b->d_tab) (void)hipFree(b->d_tab);
    if (b->h_tab) (void)hipHostFree(b->h_tab);
    if (b->uploaded) (void)hipEventDestroy(b->uploaded);
    if (b->finished) (void)hipEventDestroy(b->finished);
    delete b;
    return TX_OK;
}

}  // extern "C"
