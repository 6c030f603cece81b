// Batched frames: many independent denoiser streams of uneven sizes, one
// launch per pass over the tiles of all streams, the passes of
// a frame captured once as a HIP graph and replayed every frame.
//
// Each frame the plan runs sv_denoise_frame for every stream with a launch
// recorder installed: the same validation and argument construction as a
// single stream, but every pass launcher hands over its argument struct
// instead of launching.  The structs of all streams go to one device
// buffer (from pinned staging, double-buffered) and the graph, whose
// kernels read their arguments from that buffer, is launched.
#include <new>

#include "sv_internal.h"

namespace {

constexpr int kMaxStreams = 64;
constexpr int kMaxPasses = 64;

inline size_t align16(size_t v) { return (v + 15) & ~(size_t)15; }

}  // namespace

struct sv_batch {
    int n = 0;
    sv_dtype t = SV_F32;
    sv_frame_params p[kMaxStreams];  // per stream
    sv_dims dims[kMaxStreams];
    sv_denoiser *st[kMaxStreams];
    // pass structure, fixed by the first frame
    int npass = 0;
    sv::BatchLaunch fn[kMaxPasses];
    size_t arg_size[kMaxPasses];
    int total[kMaxPasses];
    size_t off_args[kMaxPasses], off_prefix[kMaxPasses];
    size_t bytes = 0;
    unsigned char *dev = nullptr;
    unsigned char *host[2] = {nullptr, nullptr};
    hipEvent_t ev[2] = {nullptr, nullptr};
    int parity = 0;
    bool direct = false;  // launch the passes each frame instead of replaying the graph
    bool broken = false;  // a failed allocation or capture: the plan is unusable
    hipStream_t cap = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    sv::PassRecord rec[kMaxStreams][kMaxPasses];
};

static void release(sv_batch *b) {
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    for (int i = 0; i < 2; ++i) {
        if (b->ev[i]) (void)hipEventDestroy(b->ev[i]);
        if (b->host[i]) (void)hipHostFree(b->host[i]);
    }
    if (b->dev) (void)hipFree(b->dev);
    delete b;
}

static int create(const sv_dims *dims, sv_denoiser *const *states, int32_t n, sv_dtype t,
                  const sv_frame_params *p, size_t p_stride, sv_batch **out) {
    using namespace sv;
    if (!out) return SV_EINVAL;
    *out = nullptr;
    if (!valid_dtype(t)) return SV_EDTYPE;
    if (!dims || !states || !p || n < 1 || n > kMaxStreams) return SV_EINVAL;
    for (int i = 0; i < n; ++i) {
        const sv_frame_params &pi = p[i * p_stride];
        if (pi.levels < 1 || pi.levels > 5) return SV_EUNSUPPORTED;  // steps 1..16: tiled passes
        // one level whose output is the colour history needs a separate
        // final pass; not batched
        if (pi.levels == 1 && pi.feedback != 1) return SV_EUNSUPPORTED;
        if (check_dims(dims[i]) != 0 || !states[i]) return SV_EINVAL;
        for (int j = 0; j < i; ++j)
            if (states[j] == states[i]) return SV_EALIAS;
    }
    sv_batch *b = new (std::nothrow) sv_batch();
    if (!b) return SV_EHIP;
    b->n = n;
    b->t = t;
    for (int i = 0; i < n; ++i) {
        b->p[i] = p[i * p_stride];
        b->dims[i] = dims[i];
        b->st[i] = states[i];
    }
    *out = b;
    return SV_OK;
}

extern "C" int sv_batch_create(const sv_dims *dims, sv_denoiser *const *states, int32_t n,
                               sv_dtype t, const sv_frame_params *p, sv_batch **out) {
    return create(dims, states, n, t, p, 0, out);
}

extern "C" int sv_batch_create_each(const sv_dims *dims, sv_denoiser *const *states, int32_t n,
                                    sv_dtype t, const sv_frame_params *params, sv_batch **out) {
    return create(dims, states, n, t, params, 1, out);
}

extern "C" void sv_batch_destroy(sv_batch *b) {
    if (b) release(b);
}

// Records stream i's frame; on failure the streams already recorded are
// returned to their previous history buffer.
static int record_all(sv_batch *b, const sv_frame_in *in, int counts[]) {
    using namespace sv;
    for (int i = 0; i < b->n; ++i) {
        Recorder r{b->rec[i], kMaxPasses, 0, false};
        recorder() = &r;
        const int rc = sv_denoise_frame(&in[i], b->st[i], b->dims[i], b->t, &b->p[i], nullptr);
        recorder() = nullptr;
        counts[i] = r.count;
        if (rc != SV_OK || r.overflow) {
            for (int j = 0; j < i + (rc == SV_OK ? 1 : 0); ++j) b->st[j]->cur ^= 1;
            return rc != SV_OK ? rc : SV_EUNSUPPORTED;
        }
    }
    return SV_OK;
}

static int build_plan(sv_batch *b, const int counts[]) {
    using namespace sv;
    b->npass = counts[0];
    size_t off = 0;
    for (int k = 0; k < b->npass; ++k) {
        const PassRecord &r0 = b->rec[0][k];
        if (!r0.fn) return SV_EUNSUPPORTED;
        b->fn[k] = r0.fn;
        b->arg_size[k] = r0.arg_size;
        b->off_args[k] = off;
        off = align16(off + (size_t)b->n * r0.arg_size);
        b->off_prefix[k] = off;
        off = align16(off + (size_t)(b->n + 1) * sizeof(int));
    }
    b->bytes = off;
    if (hipMalloc((void **)&b->dev, b->bytes) != hipSuccess) return SV_EHIP;
    for (int i = 0; i < 2; ++i) {
        if (hipHostMalloc((void **)&b->host[i], b->bytes, hipHostMallocDefault) != hipSuccess)
            return SV_EHIP;
        if (hipEventCreateWithFlags(&b->ev[i], hipEventDisableTiming) != hipSuccess) return SV_EHIP;
    }
    return SV_OK;
}

static int check_structure(const sv_batch *b, const int counts[]) {
    for (int i = 0; i < b->n; ++i) {
        if (counts[i] != b->npass) return SV_EINVAL;
        for (int k = 0; k < b->npass; ++k) {
            const sv::PassRecord &r = b->rec[i][k];
            if (r.fn != b->fn[k] || r.arg_size != b->arg_size[k]) return SV_EINVAL;
        }
    }
    return SV_OK;
}

static void fill(sv_batch *b, unsigned char *h) {
    for (int k = 0; k < b->npass; ++k) {
        int *prefix = (int *)(h + b->off_prefix[k]);
        prefix[0] = 0;
        for (int i = 0; i < b->n; ++i) {
            const sv::PassRecord &r = b->rec[i][k];
            unsigned char *dst = h + b->off_args[k] + (size_t)i * r.arg_size;
            for (size_t j = 0; j < r.arg_size; ++j) dst[j] = r.args[j];
            prefix[i + 1] = prefix[i] + r.tiles;
        }
        b->total[k] = prefix[b->n];
    }
}

static int capture(sv_batch *b) {
    if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) return SV_EHIP;
    if (hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
        return SV_EHIP;
    for (int k = 0; k < b->npass; ++k)
        b->fn[k](b->dev + b->off_args[k], (const int *)(b->dev + b->off_prefix[k]), b->n,
                 b->total[k], b->cap);
    const hipError_t e1 = hipGetLastError();
    const hipError_t e2 = hipStreamEndCapture(b->cap, &b->graph);
    if (e1 != hipSuccess || e2 != hipSuccess) return SV_EHIP;
    if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) return SV_EHIP;
    return SV_OK;
}

extern "C" int sv_batch_frame(sv_batch *b, const sv_frame_in *in, sv_stream stream) {
    using namespace sv;
    if (!b || !in) return SV_EINVAL;
    if (b->broken) return SV_EHIP;
    int counts[kMaxStreams];
    int rc = record_all(b, in, counts);
    if (rc != SV_OK) return rc;
    for (int i = 1; i < b->n; ++i)
        if (counts[i] != counts[0]) rc = SV_EINVAL;
    const bool first = b->exec == nullptr;
    if (rc == SV_OK && first && !b->dev) {
        rc = build_plan(b, counts);
        if (rc == SV_EHIP) b->broken = true;
    }
    if (rc == SV_OK) rc = check_structure(b, counts);
    if (rc != SV_OK) {
        for (int i = 0; i < b->n; ++i) b->st[i]->cur ^= 1;  // nothing was enqueued
        return rc;
    }
    hipStream_t s = as_stream(stream);
    // the copy that last read this staging buffer (two frames ago) is done
    if (hipEventSynchronize(b->ev[b->parity]) != hipSuccess) return SV_EHIP;
    unsigned char *h = b->host[b->parity];
    fill(b, h);
    if (hipMemcpyAsync(b->dev, h, b->bytes, hipMemcpyHostToDevice, s) != hipSuccess) return SV_EHIP;
    if (hipEventRecord(b->ev[b->parity], s) != hipSuccess) return SV_EHIP;
    b->parity ^= 1;
    if (b->direct) {  // the same passes, launched on the caller's stream
        for (int k = 0; k < b->npass; ++k)
            b->fn[k](b->dev + b->off_args[k], (const int *)(b->dev + b->off_prefix[k]), b->n,
                     b->total[k], s);
        return hip_status(hipGetLastError());
    }
    if (first) {
        rc = capture(b);
        if (rc != SV_OK) {
            b->broken = true;
            return rc;
        }
    }
    return hip_status(hipGraphLaunch(b->exec, s));
}

extern "C" int sv_batch_set_direct(sv_batch *b, int32_t direct) {
    if (!b || (direct != 0 && direct != 1)) return SV_EINVAL;
    b->direct = direct != 0;
    return SV_OK;
}

extern "C" int sv_batch_passes(const sv_batch *b) { return b ? b->npass : -1; }
