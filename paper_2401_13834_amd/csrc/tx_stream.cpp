// Streams: per-beam device history of the last `overlap` samples, so that
// consecutive blocks dedisperse exactly as their concatenation would (the
// paper's "write data" and "shift data" steps, Sec. 2.3).
#include <algorithm>
#include <new>

#include "tx_internal.h"

namespace tx {

tx_status stream_ingest(tx_stream_s* s, const uint8_t* block, int64_t block_pitch, int64_t nt, int block_on_device,
                        hipStream_t st, int64_t* n_out) {
    const tx_plan_s* p = s->plan;
    if (nt < 1 || nt > s->max_block || !block || block_pitch < nt || !n_out) return TX_EINVAL;
    const hipMemcpyKind kind = block_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    // The block goes right behind the history, at the 16-byte aligned byte
    // pad + overlap of every row.
    hipError_t e = hipMemcpy2DAsync(s->ring + s->pad + p->overlap, static_cast<size_t>(s->pitch), block,
                                    static_cast<size_t>(block_pitch), static_cast<size_t>(nt),
                                    static_cast<size_t>(p->nchan), kind, st);
    if (e != hipSuccess) return status_of(e);
    *n_out = std::max<int64_t>(0, s->held + nt - p->overlap);
    return TX_OK;
}

tx_status stream_ingest_tf(tx_stream_s* s, const uint8_t* block, int64_t block_pitch, int64_t nt,
                           int block_on_device, hipStream_t st, int64_t* n_out) {
    const tx_plan_s* p = s->plan;
    if (nt < 1 || nt > s->max_block || !block || block_pitch < p->nchan || !n_out) return TX_EINVAL;
    const uint8_t* src = block;
    int64_t src_pitch = block_pitch;
    if (block_on_device) {
        if ((reinterpret_cast<uintptr_t>(block) & 15) || (block_pitch & 15)) return TX_EINVAL;
    } else {
        if (!s->stage) {
            // Sized for the largest block; kept until close.
            const tx_status rp = retain_pool(s->device);
            if (rp != TX_OK) return rp;
            const int64_t sp = (static_cast<int64_t>(p->nchan) + 15) / 16 * 16;
            void* m = nullptr;
            const hipError_t e = hipMallocAsync(&m, static_cast<size_t>(sp * s->max_block), st);
            if (e != hipSuccess) return status_of(e);
            s->stage = static_cast<uint8_t*>(m);
            s->stage_pitch = sp;
        }
        const hipError_t e = hipMemcpy2DAsync(s->stage, static_cast<size_t>(s->stage_pitch), block,
                                              static_cast<size_t>(block_pitch), static_cast<size_t>(p->nchan),
                                              static_cast<size_t>(nt), hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return status_of(e);
        src = s->stage;
        src_pitch = s->stage_pitch;
    }
    const hipError_t e = launch_transpose_tf(src, src_pitch, p->nchan, nt, s->ring + s->pad + p->overlap, s->pitch, st);
    if (e != hipSuccess) return status_of(e);
    *n_out = std::max<int64_t>(0, s->held + nt - p->overlap);
    return TX_OK;
}

void stream_input(const tx_stream_s* s, const uint8_t** base, int* x_off) {
    const int64_t first = s->pad + s->plan->overlap - s->held;
    *base = s->ring + (first & ~int64_t(15));
    *x_off = static_cast<int>(first & 15);
}

tx_status stream_advance(tx_stream_s* s, int64_t nt, hipStream_t st) {
    const int64_t O = s->plan->overlap;
    const int64_t have = s->held + nt;
    const int64_t n_out = std::max<int64_t>(0, have - O);
    const int64_t keep = std::min(have, O);
    if (keep > 0) {
        // Move the last `keep` samples of every row back by nt, so that the
        // history ends at pad + O again (the paper's "shift data").  The copy
        // is widened at its front to a multiple of 128 bytes, so its
        // destination covers whole cache lines (the extra bytes precede the
        // history and are never read).  Source and destination overlap when
        // the shift is below the width: then copy forward in pieces no wider
        // than the shift, so no piece overwrites a source byte that a later
        // piece still reads, or, for many pieces, through a transient buffer
        // from the stream-ordered pool.
        const int64_t end = s->pad + O;
        const int64_t w = (keep + 127) & ~int64_t(127);
        uint8_t* dst = s->ring + (end - w);
        const uint8_t* src = s->ring + (end + nt - w);
        const size_t rows = static_cast<size_t>(s->plan->nchan);
        const size_t pitch = static_cast<size_t>(s->pitch);
        if (nt >= w || (w + nt - 1) / nt <= 8) {
            for (int64_t x = 0; x < w; x += nt) {
                const int64_t pw = std::min(nt, w - x);
                hipError_t e = hipMemcpy2DAsync(dst + x, pitch, src + x, pitch, static_cast<size_t>(pw), rows,
                                                hipMemcpyDeviceToDevice, st);
                if (e != hipSuccess) return status_of(e);
            }
        } else {
            void* tmp = nullptr;
            hipError_t e = hipMallocAsync(&tmp, static_cast<size_t>(w) * rows, st);
            if (e != hipSuccess) return status_of(e);
            uint8_t* t = static_cast<uint8_t*>(tmp);
            e = hipMemcpy2DAsync(t, static_cast<size_t>(w), src, pitch, static_cast<size_t>(w), rows,
                                 hipMemcpyDeviceToDevice, st);
            if (e == hipSuccess)
                e = hipMemcpy2DAsync(dst, pitch, t, static_cast<size_t>(w), static_cast<size_t>(w), rows,
                                     hipMemcpyDeviceToDevice, st);
            const hipError_t ef = hipFreeAsync(tmp, st);
            if (e == hipSuccess) e = ef;
            if (e != hipSuccess) return status_of(e);
        }
    }
    s->held = keep;
    s->received += nt;
    s->emitted += n_out;
    return TX_OK;
}

}  // namespace tx

static void free_stream(tx_stream_s* s) {
    if (s->ring || s->ws || s->stage) (void)hipDeviceSynchronize();
    if (s->ring) (void)hipFree(s->ring);
    if (s->ws || s->stage) {
        if (s->ws) (void)hipFreeAsync(s->ws, nullptr);
        if (s->stage) (void)hipFreeAsync(s->stage, nullptr);
        (void)hipStreamSynchronize(nullptr);
    }
    delete s;
}

extern "C" {

tx_status tx_stream_open(tx_plan_t plan, int64_t max_block, tx_stream_t* out) {
    if (!plan || !out || max_block < 1 || max_block > (int64_t(1) << 30)) return TX_EINVAL;
    *out = nullptr;
    if (!plan->on_device) return TX_ESTATE;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return TX_EDEVICE;
    if (dev != plan->device) return TX_ESTATE;
    const tx::DedispGeom geo = tx::dedisp_geometry(plan, max_block, tx::plan_tiles(plan));
    if (!geo.ok) return TX_ENOTSUP;
    tx_stream_s* s = new (std::nothrow) tx_stream_s();
    if (!s) return TX_ENOMEM;
    s->plan = plan;
    s->device = dev;
    s->max_block = max_block;
    s->pad = (128 - plan->overlap % 128) % 128;
    s->pitch = (s->pad + plan->overlap + max_block + 255) / 256 * 256;
    const size_t bytes = static_cast<size_t>(s->pitch) * plan->nchan;
    const hipError_t e = hipMalloc(reinterpret_cast<void**>(&s->ring), bytes);
    if (e != hipSuccess) {
        free_stream(s);
        return tx::status_of(e);
    }
    *out = s;
    return TX_OK;
}

static tx_status push_block(tx_stream_t s, const uint8_t* block, int64_t block_pitch, int64_t nt,
                            int32_t block_on_device, bool time_major, int32_t* d_out, int64_t out_pitch,
                            int64_t* nt_out, hipStream_t stream) {
    if (!s || !nt_out) return TX_EINVAL;
    tx_status st = tx::check_out_args(d_out, out_pitch, nt);
    if (st != TX_OK) return st;
    int64_t n_out = 0;
    st = time_major ? tx::stream_ingest_tf(s, block, block_pitch, nt, block_on_device, stream, &n_out)
                    : tx::stream_ingest(s, block, block_pitch, nt, block_on_device, stream, &n_out);
    if (st != TX_OK) return st;
    if (n_out > 0) {
        const tx::DedispGeom geo = tx::dedisp_geometry(s->plan, n_out, tx::plan_tiles(s->plan));
        if (!geo.ok) return TX_ENOTSUP;
        if (geo.ws_bytes > s->ws_bytes) {
            // Sized for the largest block this stream accepts; kept until close.
            const tx::DedispGeom big = tx::dedisp_geometry(s->plan, s->max_block, tx::plan_tiles(s->plan));
            const int64_t want = std::max(big.ws_bytes, geo.ws_bytes);
            if (s->ws) (void)hipFreeAsync(s->ws, stream);
            s->ws = nullptr;
            s->ws_bytes = 0;
            const tx_status rp = tx::retain_pool(s->device);
            if (rp != TX_OK) return rp;
            const hipError_t e = hipMallocAsync(&s->ws, static_cast<size_t>(want), stream);
            if (e != hipSuccess) return tx::status_of(e);
            s->ws_bytes = want;
        }
        const uint8_t* base = nullptr;
        int x_off = 0;
        tx::stream_input(s, &base, &x_off);
        const hipError_t e = tx::launch_dedisperse(s->plan, geo, base, s->pitch, n_out, d_out, out_pitch,
                                                   static_cast<uint16_t*>(s->ws), stream, x_off);
        if (e != hipSuccess) return tx::status_of(e);
    }
    st = tx::stream_advance(s, nt, stream);
    if (st != TX_OK) return st;
    *nt_out = n_out;
    return TX_OK;
}

tx_status tx_stream_push(tx_stream_t s, const uint8_t* block, int64_t block_pitch, int64_t nt, int32_t block_on_device,
                         int32_t* d_out, int64_t out_pitch, int64_t* nt_out, hipStream_t stream) {
    return push_block(s, block, block_pitch, nt, block_on_device, false, d_out, out_pitch, nt_out, stream);
}

tx_status tx_stream_push_tf(tx_stream_t s, const uint8_t* block, int64_t block_pitch, int64_t nt,
                            int32_t block_on_device, int32_t* d_out, int64_t out_pitch, int64_t* nt_out,
                            hipStream_t stream) {
    return push_block(s, block, block_pitch, nt, block_on_device, true, d_out, out_pitch, nt_out, stream);
}

tx_status tx_stream_position(tx_stream_t s, int64_t* received, int64_t* emitted) {
    if (!s || !received || !emitted) return TX_EINVAL;
    *received = s->received;
    *emitted = s->emitted;
    return TX_OK;
}

tx_status tx_stream_reset(tx_stream_t s) {
    if (!s) return TX_EINVAL;
    s->held = 0;
    s->received = 0;
    s->emitted = 0;
    return TX_OK;
}

tx_status tx_stream_snapshot(tx_stream_t s, uint8_t* host_hist, int64_t* held, int64_t* received, int64_t* emitted,
                             hipStream_t stream) {
    if (!s || !held || !received || !emitted || (s->held > 0 && !host_hist)) return TX_EINVAL;
    if (s->held > 0) {
        const int64_t first = s->pad + s->plan->overlap - s->held;
        hipError_t e = hipMemcpy2DAsync(host_hist, static_cast<size_t>(s->held), s->ring + first,
                                        static_cast<size_t>(s->pitch), static_cast<size_t>(s->held),
                                        static_cast<size_t>(s->plan->nchan), hipMemcpyDeviceToHost, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return tx::status_of(e);
    }
    *held = s->held;
    *received = s->received;
    *emitted = s->emitted;
    return TX_OK;
}

tx_status tx_stream_restore(tx_stream_t s, const uint8_t* host_hist, int64_t held, int64_t received, int64_t emitted,
                            hipStream_t stream) {
    if (!s || held < 0 || held > s->plan->overlap || received < held || emitted < 0 || (held > 0 && !host_hist))
        return TX_EINVAL;
    if (received != emitted + held) return TX_EINVAL;
    if (held > 0) {
        const int64_t first = s->pad + s->plan->overlap - held;
        hipError_t e = hipMemcpy2DAsync(s->ring + first, static_cast<size_t>(s->pitch), host_hist,
                                        static_cast<size_t>(held), static_cast<size_t>(held),
                                        static_cast<size_t>(s->plan->nchan), hipMemcpyHostToDevice, stream);
        if (e == hipSuccess) e = hipStreamSynchronize(stream);
        if (e != hipSuccess) return tx::status_of(e);
    }
    s->held = held;
    s->received = received;
    s->emitted = emitted;
    return TX_OK;
}

tx_status tx_stream_close(tx_stream_t s) {
    if (!s) return TX_OK;
    free_stream(s);
    return TX_OK;
}

}  // extern "C"
