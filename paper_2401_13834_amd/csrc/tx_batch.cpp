// Batches: the jobs of many beams (uneven channel counts, block lengths and DM
// grids) run as one persistent launch per stage, optionally captured in a HIP
// graph.  The job tables live in device memory and are refreshed before every
// launch, so a captured graph can be replayed over a different set of jobs.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "tx_internal.h"

namespace {

constexpr int kIWs[] = {16, 13, 8, 4, 2, 1};
constexpr int kNIW = 6;

int iw_index(int iw) {
    for (int k = 0; k < kNIW; ++k)
        if (kIWs[k] == iw) return k;
    return -1;
}

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

// Layout of the integer table: prefix sums and job counts of every launch.
struct IntLayout {
    int max_jobs;
    int p1() const { return 0; }
    int n1() const { return max_jobs + 1; }
    int p2(int g) const { return max_jobs + 2 + g * (max_jobs + 2); }
    int n2(int g) const { return p2(g) + max_jobs + 1; }
    int pb() const { return p2(kNIW); }
    int nb() const { return pb() + max_jobs + 1; }
    int size() const { return nb() + 1; }
};

struct Signature {            // what a captured graph bakes in
    int s1 = -1, lds1 = 0, s2 = -1, lds2 = 0;
    bool groups[kNIW] = {};
    int nwt = 0;
    int ldsb = 0;             // boxcar dynamic LDS (per-(tile, width) maxima)
    bool any_box = false;
    // grids: first-stage tiles, second-stage tiles per group, boxcar rows
    int64_t g1 = 0, g2[kNIW] = {}, gb = 0;
};

struct GraphSlot {
    int cap_jobs = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    Signature sig;
};

}  // namespace

struct tx_batch_s {
    int device = -1;
    int max_jobs = 0;
    uint32_t flags = 0;
    std::vector<Job> jobs;
    IntLayout L{0};
    // device tables and their pinned host mirror (one contiguous block)
    size_t off_s1 = 0, off_s2 = 0, off_bx = 0, off_int = 0, table_bytes = 0;
    uint8_t* d_tab = nullptr;
    uint8_t* h_tab = nullptr;
    hipEvent_t uploaded = nullptr;     // the last upload from h_tab has been consumed
    bool upload_pending = false;
    // first-stage series of every job of a launch
    void* scratch = nullptr;
    int64_t scratch_bytes = 0;
    // captured graphs, one per size class (jobs per launch, a power of two,
    // when plans were reserved; a single class otherwise)
    std::vector<GraphSlot> graphs;
    // plans declared ahead of the first launch (tx_batch_reserve): the union
    // of their kernels and LDS sizes, and the largest grids of one job
    bool reserved = false;
    Signature floor;
    tx::Tiles tiles{};
};

namespace {

void destroy_graphs(tx_batch_s* b) {
    for (GraphSlot& g : b->graphs) {
        if (g.exec) (void)hipGraphExecDestroy(g.exec);
        if (g.graph) (void)hipGraphDestroy(g.graph);
    }
    b->graphs.clear();
}

// Size class of a launch of n jobs: the next power of two (at most max_jobs)
// when plans were reserved, so that small launches replay small grids.
int size_class(const tx_batch_s* b, int n) {
    if (!b->reserved) return b->max_jobs;
    int c = 1;
    while (c < n) c <<= 1;
    return std::min(c, b->max_jobs);
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

// Kernel launches of one batch launch (captured or direct).
hipError_t run_kernels(tx_batch_s* b, const Signature& sig, hipStream_t st) {
    const int* ints = reinterpret_cast<const int*>(b->d_tab + b->off_int);
    const tx::Stage1Args* s1 = reinterpret_cast<const tx::Stage1Args*>(b->d_tab + b->off_s1);
    const tx::Stage2Args* s2 = reinterpret_cast<const tx::Stage2Args*>(b->d_tab + b->off_s2);
    const tx::BoxcarArgs* bx = reinterpret_cast<const tx::BoxcarArgs*>(b->d_tab + b->off_bx);
    hipError_t e = hipSuccess;
    if (sig.any_box) {
        e = tx::launch_zero_counts(bx, ints + b->L.nb(), b->max_jobs, st);
        if (e != hipSuccess) return e;
    }
    e = tx::launch_stage1_batch(sig.s1, sig.lds1, s1, ints + b->L.p1(), ints + b->L.n1(), static_cast<int>(sig.g1),
                                st);
    if (e != hipSuccess) return e;
    for (int g = 0; g < kNIW; ++g) {
        if (!sig.groups[g]) continue;
        e = tx::launch_stage2_batch(kIWs[g], sig.s2, sig.lds2, s2 + static_cast<size_t>(g) * b->max_jobs,
                                    ints + b->L.p2(g), ints + b->L.n2(g), static_cast<int>(sig.g2[g]), st);
        if (e != hipSuccess) return e;
    }
    if (sig.any_box)
        e = tx::launch_boxcar_batch(sig.nwt, sig.ldsb, bx, ints + b->L.pb(), ints + b->L.nb(), static_cast<int>(sig.gb),
                                    st);
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
    b->L = IntLayout{max_jobs};
    auto align = [](size_t v) { return (v + 255) / 256 * 256; };
    b->off_s1 = 0;
    b->off_s2 = align(sizeof(tx::Stage1Args) * max_jobs);
    b->off_bx = b->off_s2 + align(sizeof(tx::Stage2Args) * max_jobs * kNIW);
    b->off_int = b->off_bx + align(sizeof(tx::BoxcarArgs) * max_jobs);
    b->table_bytes = b->off_int + align(sizeof(int) * b->L.size());
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&b->d_tab), b->table_bytes);
    if (e == hipSuccess) e = hipHostMalloc(reinterpret_cast<void**>(&b->h_tab), b->table_bytes);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->uploaded, hipEventDisableTiming);
    if (e != hipSuccess) {
        tx_batch_destroy(b);
        return tx::status_of(e);
    }
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
    const tx::Tiles t = tx::plan_tiles(plan);
    if (b->reserved && (t.s1 != b->tiles.s1 || t.s2 != b->tiles.s2)) return TX_EINVAL;
    const tx::DedispGeom g = tx::dedisp_geometry(plan, max_nt, t);
    if (!g.ok) return TX_ENOTSUP;
    tx::Stage1Args a1;
    tx::Stage2Args a2;
    tx::fill_stage_args(plan, g, nullptr, max_nt + plan->overlap, max_nt, nullptr, max_nt + 1, nullptr, &a1, &a2);
    Signature f = b->floor;
    f.s1 = g.tiles.s1;
    f.s2 = g.tiles.s2;
    f.lds1 = std::max(f.lds1, g.lds1);
    f.lds2 = std::max(f.lds2, g.lds2);
    const int gi = iw_index(g.iw);
    f.groups[gi] = true;
    // grids of one job (a launch of n jobs is sized n times these)
    f.g1 = std::max(f.g1, tx::stage1_tiles(a1));
    f.g2[gi] = std::max(f.g2[gi], tx::stage2_tiles(a2));
    if (nw > 0) {
        f.any_box = true;
        f.nwt = std::max(f.nwt, tx::boxcar_nwt(nw));
        f.ldsb = std::max(f.ldsb, tx::boxcar_tmax_bytes(f.nwt, max_nt));
        f.gb = std::max<int64_t>(f.gb, plan->ndm);
    }
    const int64_t m = b->max_jobs;
    if (f.g1 * m > INT32_MAX || f.g2[gi] * m > INT32_MAX || f.gb * m > INT32_MAX) return TX_ENOTSUP;
    (void)count;
    b->floor = f;
    b->tiles = t;
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

    // Tile choice: the reserved plans, else the first job's plan, decide the
    // variants; every job's LDS need (and every reserved plan's) raises the
    // batch's LDS sizes.
    const tx::Tiles t0 = b->reserved ? b->tiles : tx::plan_tiles(b->jobs[0].plan);
    Signature sig = b->reserved ? b->floor : Signature{};
    std::vector<tx::DedispGeom> geo(static_cast<size_t>(n));
    // Stream jobs: copy the blocks behind the held histories first.
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
    int64_t scratch_need = 0;
    std::vector<int64_t> scratch_off(static_cast<size_t>(n), 0);
    for (int k = 0; k < n; ++k) {
        Job& j = b->jobs[static_cast<size_t>(k)];
        geo[static_cast<size_t>(k)] = tx::dedisp_geometry(j.plan, std::max<int64_t>(j.nt_out, 1), t0);
        const tx::DedispGeom& g = geo[static_cast<size_t>(k)];
        if (!g.ok) return TX_ENOTSUP;
        sig.s1 = g.tiles.s1;
        sig.s2 = g.tiles.s2;
        sig.lds1 = std::max(sig.lds1, g.lds1);
        sig.lds2 = std::max(sig.lds2, g.lds2);
        sig.groups[iw_index(g.iw)] = true;   // by plan, so a graph captured while priming still fits
        if (j.has_box) {
            sig.any_box = true;
            sig.nwt = std::max(sig.nwt, tx::boxcar_nwt(j.box.nw));
        }
        if (j.nt_out > 0) {
            scratch_off[static_cast<size_t>(k)] = scratch_need;
            scratch_need += g.ws_bytes;
        }
    }
    // Grids: the tiles and rows of this launch.
    int64_t tot1 = 0, tot2[kNIW] = {}, totb = 0;
    for (int k = 0; k < n; ++k) {
        const Job& j = b->jobs[static_cast<size_t>(k)];
        if (j.nt_out <= 0) continue;
        tx::Stage1Args a1;
        tx::Stage2Args a2;
        tx::fill_stage_args(j.plan, geo[static_cast<size_t>(k)], nullptr, 0, j.nt_out, nullptr, 0, nullptr, &a1, &a2);
        tot1 += tx::stage1_tiles(a1);
        tot2[iw_index(geo[static_cast<size_t>(k)].iw)] += tx::stage2_tiles(a2);
        if (j.has_box) totb += j.plan->ndm;
    }
    // Boxcar dynamic LDS: the per-(tile, width) maxima of the longest row that
    // fits (longer rows rescan their tiles instead).
    int ldsb = 0;
    for (const Job& j : b->jobs)
        if (j.has_box && j.nt_out > 0) ldsb = std::max(ldsb, tx::boxcar_tmax_bytes(sig.nwt, j.nt_out));
    const bool use_graph = (b->flags & TX_BATCH_GRAPH) && stream != nullptr;
    const int cls = size_class(b, n);
    GraphSlot* slot = nullptr;
    if (use_graph)
        for (GraphSlot& g : b->graphs)
            if (g.cap_jobs == cls) slot = &g;
    if (slot) {
        // A captured graph fixes the kernels, grids and LDS sizes.
        Signature want = slot->sig;
        bool fits = sig.s1 == want.s1 && sig.s2 == want.s2 && sig.lds1 <= want.lds1 && sig.lds2 <= want.lds2 &&
                    sig.nwt <= want.nwt && (!sig.any_box || want.any_box) && tot1 <= want.g1 && totb <= want.gb;
        for (int g = 0; g < kNIW; ++g)
            if ((sig.groups[g] && !want.groups[g]) || tot2[g] > want.g2[g]) fits = false;
        if (!fits) return TX_ESTATE;
        sig = want;
    } else {
        // Direct launches use the exact grids.  A graph captured now is sized
        // for its size class from the reserved plans (else for this launch,
        // with every stream job counted at its largest block).
        Signature f = b->floor;
        f.g1 *= cls;
        f.gb *= cls;
        for (int g = 0; g < kNIW; ++g) f.g2[g] *= cls;
        if (use_graph && !b->reserved) {
            int64_t c1 = 0, c2[kNIW] = {}, cb = 0;
            for (int k = 0; k < n; ++k) {
                const Job& j = b->jobs[static_cast<size_t>(k)];
                const int64_t nt_cap = j.stream ? std::max(j.stream->max_block, j.nt_out) : j.nt_out;
                if (nt_cap <= 0) continue;
                const tx::DedispGeom gc = tx::dedisp_geometry(j.plan, nt_cap, t0);
                if (!gc.ok) return TX_ENOTSUP;
                tx::Stage1Args a1;
                tx::Stage2Args a2;
                tx::fill_stage_args(j.plan, gc, nullptr, 0, nt_cap, nullptr, 0, nullptr, &a1, &a2);
                c1 += tx::stage1_tiles(a1);
                c2[iw_index(gc.iw)] += tx::stage2_tiles(a2);
                if (j.has_box) {
                    cb += j.plan->ndm;
                    ldsb = std::max(ldsb, tx::boxcar_tmax_bytes(sig.nwt, nt_cap));
                }
            }
            tot1 = std::max(tot1, c1);
            totb = std::max(totb, cb);
            for (int g = 0; g < kNIW; ++g) tot2[g] = std::max(tot2[g], c2[g]);
        }
        sig.g1 = std::max(tot1, use_graph ? f.g1 : 0);
        sig.gb = std::max(totb, use_graph ? f.gb : 0);
        sig.ldsb = std::max(ldsb, use_graph ? f.ldsb : 0);
        for (int g = 0; g < kNIW; ++g) sig.g2[g] = std::max(tot2[g], use_graph ? f.g2[g] : 0);
        if (sig.g1 > INT32_MAX || sig.gb > INT32_MAX) return TX_ENOTSUP;
        for (int g = 0; g < kNIW; ++g)
            if (sig.g2[g] > INT32_MAX) return TX_ENOTSUP;
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
    // Job tables into the pinned mirror (after the previous upload was consumed).
    if (b->upload_pending) {
        const hipError_t e = hipEventSynchronize(b->uploaded);
        if (e != hipSuccess) return tx::status_of(e);
        b->upload_pending = false;
    }
    auto* h1 = reinterpret_cast<tx::Stage1Args*>(b->h_tab + b->off_s1);
    auto* h2 = reinterpret_cast<tx::Stage2Args*>(b->h_tab + b->off_s2);
    auto* hb = reinterpret_cast<tx::BoxcarArgs*>(b->h_tab + b->off_bx);
    int* hi = reinterpret_cast<int*>(b->h_tab + b->off_int);
    int n1 = 0, nb = 0;
    int n2[kNIW] = {};
    hi[b->L.p1()] = 0;
    for (int g = 0; g < kNIW; ++g) hi[b->L.p2(g)] = 0;
    hi[b->L.pb()] = 0;
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
        a1.lds_bytes = sig.lds1;
        a2.lds_bytes = sig.lds2;
        h1[n1] = a1;
        hi[b->L.p1() + n1 + 1] = hi[b->L.p1() + n1] + static_cast<int>(tx::stage1_tiles(a1));
        ++n1;
        const int gi = iw_index(g.iw);
        h2[static_cast<size_t>(gi) * b->max_jobs + n2[gi]] = a2;
        hi[b->L.p2(gi) + n2[gi] + 1] = hi[b->L.p2(gi) + n2[gi]] + static_cast<int>(tx::stage2_tiles(a2));
        ++n2[gi];
        if (j.has_box) {
            tx::BoxcarArgs bx = j.box;
            bx.y = j.out;
            bx.pitch = j.out_pitch;
            bx.ndm = j.plan->ndm;
            bx.nt = static_cast<int32_t>(j.nt_out);
            tx::boxcar_fit(&bx, j.box.widths, j.box.nw, j.nt_out);
            const int need = tx::boxcar_tmax_bytes(sig.nwt, j.nt_out);
            bx.tmax_ok = (need > 0 && need <= sig.ldsb) ? 1 : 0;
            hb[nb] = bx;
            hi[b->L.pb() + nb + 1] = hi[b->L.pb() + nb] + bx.ndm;
            ++nb;
        }
    }
    hi[b->L.n1()] = n1;
    for (int g = 0; g < kNIW; ++g) hi[b->L.n2(g)] = n2[g];
    hi[b->L.nb()] = nb;
    hipError_t e = hipMemcpyAsync(b->d_tab, b->h_tab, b->table_bytes, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess) e = hipEventRecord(b->uploaded, stream);
    if (e != hipSuccess) return tx::status_of(e);
    b->upload_pending = true;

    // Kernels.
    if (use_graph) {
        if (!slot) {
            GraphSlot ns;
            ns.cap_jobs = cls;
            ns.sig = sig;
            e = hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal);
            if (e == hipSuccess) {
                const hipError_t ek = run_kernels(b, sig, stream);
                hipGraph_t g = nullptr;
                e = hipStreamEndCapture(stream, &g);
                if (ek != hipSuccess) e = ek;
                if (e == hipSuccess) {
                    ns.graph = g;
                    e = hipGraphInstantiate(&ns.exec, g, nullptr, nullptr, 0);
                } else if (g) {
                    (void)hipGraphDestroy(g);
                }
            }
            if (e != hipSuccess) {
                if (ns.exec) (void)hipGraphExecDestroy(ns.exec);
                if (ns.graph) (void)hipGraphDestroy(ns.graph);
                return tx::status_of(e);
            }
            b->graphs.push_back(ns);
            slot = &b->graphs.back();
        }
        e = hipGraphLaunch(slot->exec, stream);
    } else {
        e = run_kernels(b, sig, stream);
    }
    if (e != hipSuccess) return tx::status_of(e);
    // Stream jobs: keep the last `overlap` samples.
    for (Job& j : b->jobs) {
        if (!j.stream) continue;
        const tx_status st = tx::stream_advance(j.stream, j.nt, stream);
        if (st != TX_OK) return st;
    }
    return TX_OK;
}

tx_status tx_batch_destroy(tx_batch_t b) {
    if (!b) return TX_OK;
    if (b->upload_pending) (void)hipEventSynchronize(b->uploaded);
    destroy_graphs(b);
    if (b->scratch) {
        (void)hipDeviceSynchronize();
        (void)hipFreeAsync(b->scratch, nullptr);
        (void)hipStreamSynchronize(nullptr);
    }
    if (b->d_tab) (void)hipFree(b->d_tab);
    if (b->h_tab) (void)hipHostFree(b->h_tab);
    if (b->uploaded) (void)hipEventDestroy(b->uploaded);
    delete b;
    return TX_OK;
}

}  // extern "C"
