// lbk_batch.hip -- host side of the ensemble calls in include/lbk.h: the
// tile list over every sample, the per-sample descriptor tables, graph
// recording of step runs and the launch-configuration tuner.  The kernels
// are the batched forms in lbk_kernels.hip.
#include "lbk_host.h"

#include <math.h>
#include <string.h>

#include <new>
#include <vector>

using namespace lbk;

namespace {

constexpr int kMaxSamples = 1 << 20;
constexpr int kMaxGrid = 1 << 20;
constexpr int kMaxGraphSteps = 1024;
constexpr int kMaxRows = 64;

// Tile shape: tile_x consecutive x (the workgroup size) by `rows` rows.
struct Shape {
    int tile_x, rows;
};
constexpr Shape kReadShape{kBlock, 1}; // the batched read-out's tiling
constexpr Shape kFinest{64, 1};        // most tiles of any allowed shape

bool valid_shape(int tile_x, int rows)
{
    return tile_x >= 64 && tile_x <= kBatchMaxTile && (tile_x & 63) == 0 && rows >= 1 &&
           rows <= kMaxRows;
}

int tiles_per_row(int nx, int tile_x) { return (nx + tile_x - 1) / tile_x; }

int64_t tiles_of(const lbk_lattice *l, Shape sh)
{
    return (int64_t)tiles_per_row(l->d.nx, sh.tile_x) * ((l->d.ny + sh.rows - 1) / sh.rows);
}

int64_t total_tiles(lbk_lattice *const *lats, int n, Shape sh)
{
    int64_t t = 0;
    for (int i = 0; i < n; ++i)
        t += tiles_of(lats[i], sh);
    return t;
}

// Workspace regions: descriptor table and tile -> sample map of the sweep
// (sized for the finest allowed tiling) and of the read-out; read-out
// partials [MAC_SLOTS][read tiles] and per-sample sums [n][MAC_SLOTS].
struct BatchLayout {
    size_t desc_sweep, map_sweep, desc_read, map_read;
    int64_t max_sweep_tiles, read_tiles;
    size_t partials, results, total;
};

lbk_status check_lattices(lbk_lattice *const *lats, int n)
{
    if (!lats)
        return fail(LBK_ERR_INVALID_ARG, "lats is NULL");
    if (n < 1 || n > kMaxSamples)
        return fail(LBK_ERR_INVALID_ARG, "need 1 <= n <= %d samples (got %d)", kMaxSamples, n);
    for (int i = 0; i < n; ++i) {
        const lbk_lattice *l = lats[i];
        if (!l)
            return fail(LBK_ERR_INVALID_ARG, "lats[%d] is NULL", i);
        for (int j = 0; j < i; ++j)
            if (lats[j] == l)
                return fail(LBK_ERR_INVALID_ARG, "lats[%d] repeats lats[%d]", i, j);
        if (l->d.storage != lats[0]->d.storage || l->d.bc_x != lats[0]->d.bc_x ||
            l->d.bc_y != lats[0]->d.bc_y)
            return fail(LBK_ERR_UNSUPPORTED,
                        "sample %d differs from sample 0 in storage or boundary kinds", i);
        if (l->stream != lats[0]->stream)
            return fail(LBK_ERR_INVALID_ARG, "sample %d was created on another stream", i);
    }
    return LBK_OK;
}

BatchLayout batch_layout(lbk_lattice *const *lats, int n)
{
    BatchLayout B{};
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes, 256);
        return at;
    };
    B.max_sweep_tiles = total_tiles(lats, n, kFinest);
    B.read_tiles = total_tiles(lats, n, kReadShape);
    B.desc_sweep = take((size_t)n * sizeof(SampleDesc));
    B.map_sweep = take((size_t)B.max_sweep_tiles * sizeof(int));
    B.desc_read = take((size_t)n * sizeof(SampleDesc));
    B.map_read = take((size_t)B.read_tiles * sizeof(int));
    B.partials = take((size_t)MAC_SLOTS * (size_t)B.read_tiles * sizeof(double));
    B.results = take((size_t)n * MAC_SLOTS * sizeof(double));
    B.total = o;
    return B;
}

} // namespace

struct lbk_batch {
    std::vector<lbk_lattice *> lats;
    int n;
    BatchLayout B;
    char *ws;
    hipStream_t stream; // the lattices' stream
    hipStream_t cap;    // private stream used only to record graphs
    int cus;            // compute units of the device
    int parity;         // sample i's current level is state[parity] of its descriptor
    std::vector<int> cur0, scale0;
    Shape shape;        // sweep tiling
    int64_t sweep_tiles;
    std::vector<int64_t> tile0_sweep, tile0_read;
    SampleDesc *host_desc; // pinned staging, [2][n]: sweep, read-out
    double *host_res;      // pinned, [n][MAC_SLOTS]
    int grid, graph_steps;
    hipGraphExec_t exec[2]; // graphs starting at parity 0 / 1
    bool have_exec[2];

    SampleDesc *desc_sweep() const { return reinterpret_cast<SampleDesc *>(ws + B.desc_sweep); }
    SampleDesc *desc_read() const { return reinterpret_cast<SampleDesc *>(ws + B.desc_read); }
    int *map_sweep() const { return reinterpret_cast<int *>(ws + B.map_sweep); }
    int *map_read() const { return reinterpret_cast<int *>(ws + B.map_read); }
    double *partials() const { return reinterpret_cast<double *>(ws + B.partials); }
    double *results() const { return reinterpret_cast<double *>(ws + B.results); }
    const lbk_desc &d0() const { return lats[0]->d; }
};

namespace {

void drop_graphs(lbk_batch *b)
{
    for (int p = 0; p < 2; ++p)
        if (b->have_exec[p]) {
            (void)hipGraphExecDestroy(b->exec[p]);
            b->have_exec[p] = false;
        }
}

// Upload the tile -> sample map of tiling `sh` into `map`; tile0[i] gets
// the first tile of sample i.  Synchronous.
lbk_status upload_map(lbk_batch *b, Shape sh, int *map, std::vector<int64_t> &tile0,
                      int64_t &ntiles)
{
    std::vector<int> h;
    h.reserve((size_t)total_tiles(b->lats.data(), b->n, sh));
    tile0.assign(b->n, 0);
    for (int i = 0; i < b->n; ++i) {
        tile0[i] = (int64_t)h.size();
        h.insert(h.end(), (size_t)tiles_of(b->lats[i], sh), i);
    }
    ntiles = (int64_t)h.size();
    HIP_TRY(hipStreamSynchronize(b->stream));
    HIP_TRY(hipMemcpy(map, h.data(), h.size() * sizeof(int), hipMemcpyHostToDevice));
    return LBK_OK;
}

// Bring the device descriptor tables in line with the lattices: a lattice
// stepped, loaded or rescaled outside the batch changes which of its levels
// is current or its FP16 scale.
lbk_status sync_tables(lbk_batch *b, bool force)
{
    bool stale = force;
    for (int i = 0; i < b->n && !stale; ++i) {
        const lbk_lattice *l = b->lats[i];
        stale = l->cur != (b->cur0[i] ^ b->parity) || l->scale_exp != b->scale0[i];
    }
    if (!stale)
        return LBK_OK;
    HIP_TRY(hipStreamSynchronize(b->stream)); // staging may still feed a copy
    for (int i = 0; i < b->n; ++i) {
        lbk_lattice *l = b->lats[i];
        b->cur0[i] = l->cur ^ b->parity;
        b->scale0[i] = l->scale_exp;
        for (int k = 0; k < 2; ++k) {
            const Shape sh = k == 0 ? b->shape : kReadShape;
            SampleDesc &sd = b->host_desc[(size_t)k * b->n + i];
            sd.state[b->parity] = l->state(l->cur);
            sd.state[b->parity ^ 1] = l->state(l->cur ^ 1);
            sd.med = l->med();
            sd.lay = l->L.lay;
            sd.mlay = l->L.mlay;
            sd.g = l->g;
            sd.ph = l->ph;
            sd.s = l->s();
            sd.inv_s = l->inv_s();
            sd.tile0 = (int)(k == 0 ? b->tile0_sweep[i] : b->tile0_read[i]);
            sd.tpr = tiles_per_row(l->d.nx, sh.tile_x);
        }
    }
    HIP_TRY(hipMemcpyAsync(b->desc_sweep(), b->host_desc, (size_t)b->n * sizeof(SampleDesc),
                           hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipMemcpyAsync(b->desc_read(), b->host_desc + b->n, (size_t)b->n * sizeof(SampleDesc),
                           hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    return LBK_OK;
}

// Switch the sweep to tiling `sh` (map and descriptors).
lbk_status set_shape(lbk_batch *b, Shape sh)
{
    if (sh.tile_x == b->shape.tile_x && sh.rows == b->shape.rows && b->sweep_tiles > 0)
        return LBK_OK;
    drop_graphs(b);
    b->shape = sh;
    lbk_status s = upload_map(b, sh, b->map_sweep(), b->tile0_sweep, b->sweep_tiles);
    if (s != LBK_OK)
        return s;
    return sync_tables(b, true);
}

hipError_t sweep_once(lbk_batch *b, int parity, int grid, hipStream_t st)
{
    const lbk_desc &d = b->d0();
    return launch_batch_sweep(d.storage, d.bc_x, d.bc_y, b->desc_sweep(), b->map_sweep(),
                              (int)b->sweep_tiles, parity, b->shape.tile_x, b->shape.rows, grid,
                              st);
}

// Record graph_steps launches starting at `parity` on the private stream.
lbk_status record_graph(lbk_batch *b, int parity)
{
    HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int i = 0; i < b->graph_steps && e == hipSuccess; ++i)
        e = sweep_once(b, parity ^ (i & 1), b->grid, b->cap);
    hipGraph_t graph = nullptr;
    const hipError_t e2 = hipStreamEndCapture(b->cap, &graph);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (graph)
            (void)hipGraphDestroy(graph);
        return fail(LBK_ERR_DEVICE, "graph capture: %s",
                    hipGetErrorString(e != hipSuccess ? e : e2));
    }
    e = hipGraphInstantiate(&b->exec[parity], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess)
        return fail(LBK_ERR_DEVICE, "graph instantiate: %s", hipGetErrorString(e));
    b->have_exec[parity] = true;
    return LBK_OK;
}

void destroy_batch(lbk_batch *b)
{
    drop_graphs(b);
    if (b->cap)
        (void)hipStreamDestroy(b->cap);
    if (b->host_desc)
        (void)hipHostFree(b->host_desc);
    if (b->host_res)
        (void)hipHostFree(b->host_res);
    delete b;
}

} // namespace

extern "C" {

lbk_status lbk_batch_workspace_size(lbk_lattice *const *lats, int32_t n, size_t *bytes)
{
    lbk_status s = check_lattices(lats, n);
    if (s != LBK_OK)
        return s;
    if (!bytes)
        return fail(LBK_ERR_INVALID_ARG, "bytes is NULL");
    *bytes = batch_layout(lats, n).total;
    return LBK_OK;
}

lbk_status lbk_batch_create(lbk_lattice *const *lats, int32_t n, void *workspace,
                            size_t ws_bytes, lbk_batch **out)
{
    if (!out)
        return fail(LBK_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    lbk_status s = check_lattices(lats, n);
    if (s != LBK_OK)
        return s;
    if (!workspace || ((uintptr_t)workspace & 255u))
        return fail(LBK_ERR_INVALID_ARG, "workspace must be non-NULL and 256-byte aligned");
    const BatchLayout B = batch_layout(lats, n);
    if (ws_bytes < B.total)
        return fail(LBK_ERR_OOM, "batch workspace of %zu bytes < %zu needed", ws_bytes, B.total);
    if (B.max_sweep_tiles >= ((int64_t)1 << 31))
        return fail(LBK_ERR_UNSUPPORTED, "batch of %lld tiles exceeds 2^31",
                    (long long)B.max_sweep_tiles);
    int dev = -1, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        return fail(LBK_ERR_DEVICE, "no HIP device");

    lbk_batch *b = new (std::nothrow) lbk_batch();
    if (!b)
        return fail(LBK_ERR_OOM, "host allocation failed");
    b->lats.assign(lats, lats + n);
    b->n = n;
    b->B = B;
    b->ws = static_cast<char *>(workspace);
    b->stream = lats[0]->stream;
    b->cus = cus;
    b->parity = 0;
    b->cur0.assign(n, 0);
    b->scale0.assign(n, 0);
    b->shape = Shape{0, 0};
    b->sweep_tiles = 0;
    b->grid = 0;
    b->graph_steps = 0;
    int64_t read_tiles = 0;
    if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess ||
        hipHostMalloc((void **)&b->host_desc, (size_t)2 * n * sizeof(SampleDesc),
                      hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&b->host_res, (size_t)n * MAC_SLOTS * sizeof(double),
                      hipHostMallocDefault) != hipSuccess) {
        destroy_batch(b);
        return fail(LBK_ERR_DEVICE, "stream or pinned host allocation failed");
    }
    if ((s = upload_map(b, kReadShape, b->map_read(), b->tile0_read, read_tiles)) != LBK_OK ||
        (s = set_shape(b, Shape{kBlock, 1})) != LBK_OK) {
        destroy_batch(b);
        return s;
    }
    *out = b;
    return LBK_OK;
}

lbk_status lbk_batch_destroy(lbk_batch *b)
{
    if (b)
        destroy_batch(b);
    return LBK_OK;
}

lbk_status lbk_batch_step(lbk_batch *b, int64_t n)
{
    if (!b)
        return fail(LBK_ERR_INVALID_ARG, "batch is NULL");
    if (n < 0)
        return fail(LBK_ERR_INVALID_ARG, "n must be >= 0");
    lbk_status s = sync_tables(b, false);
    if (s != LBK_OK)
        return s;
    int64_t left = n;
    while (left > 0) {
        if (b->graph_steps > 0 && left >= b->graph_steps) {
            if (!b->have_exec[b->parity] && (s = record_graph(b, b->parity)) != LBK_OK)
                return s;
            HIP_TRY(hipGraphLaunch(b->exec[b->parity], b->stream));
            left -= b->graph_steps; // even: the parity is unchanged
        } else {
            HIP_TRY(sweep_once(b, b->parity, b->grid, b->stream));
            b->parity ^= 1;
            --left;
        }
    }
    for (int i = 0; i < b->n; ++i) {
        lbk_lattice *l = b->lats[i];
        l->cur = b->cur0[i] ^ b->parity;
        l->t += n;
    }
    return LBK_OK;
}

lbk_status lbk_batch_set_launch(lbk_batch *b, int32_t tile_x, int32_t rows, int32_t grid,
                                int32_t graph_steps)
{
    if (!b)
        return fail(LBK_ERR_INVALID_ARG, "batch is NULL");
    if (!valid_shape(tile_x, rows))
        return fail(LBK_ERR_INVALID_ARG,
                    "tile_x must be 64, 128, 192 or 256 and rows 1..%d (got %d, %d)", kMaxRows,
                    tile_x, rows);
    if (grid < 0 || grid > kMaxGrid)
        return fail(LBK_ERR_INVALID_ARG, "grid must be 0..%d (got %d)", kMaxGrid, grid);
    if (graph_steps < 0 || graph_steps > kMaxGraphSteps || (graph_steps & 1))
        return fail(LBK_ERR_INVALID_ARG, "graph_steps must be 0 or even in 2..%d (got %d)",
                    kMaxGraphSteps, graph_steps);
    lbk_status s = set_shape(b, Shape{tile_x, rows});
    if (s != LBK_OK)
        return s;
    if (grid != b->grid || graph_steps != b->graph_steps)
        drop_graphs(b);
    b->grid = grid;
    b->graph_steps = graph_steps;
    return LBK_OK;
}

lbk_status lbk_batch_get_launch(const lbk_batch *b, int32_t *tile_x, int32_t *rows,
                                int32_t *grid, int32_t *graph_steps)
{
    if (!b)
        return fail(LBK_ERR_INVALID_ARG, "batch is NULL");
    if (tile_x)
        *tile_x = b->shape.tile_x;
    if (rows)
        *rows = b->shape.rows;
    if (grid)
        *grid = b->grid;
    if (graph_steps)
        *graph_steps = b->graph_steps;
    return LBK_OK;
}

lbk_status lbk_batch_autotune(lbk_batch *b, int32_t reps, double *best_us)
{
    if (!b)
        return fail(LBK_ERR_INVALID_ARG, "batch is NULL");
    if (reps < 1)
        return fail(LBK_ERR_INVALID_ARG, "reps must be >= 1");
    lbk_status s = sync_tables(b, false);
    if (s != LBK_OK)
        return s;
    hipEvent_t ev[2];
    HIP_TRY(hipEventCreate(&ev[0]));
    if (hipEventCreate(&ev[1]) != hipSuccess) {
        (void)hipEventDestroy(ev[0]);
        return fail(LBK_ERR_DEVICE, "event creation failed");
    }
    const int widths[3] = {64, 128, 256}, row_opts[4] = {1, 4, 8, 16}, per_cu[4] = {0, 2, 4, 8};
    double best = INFINITY;
    Shape best_shape = b->shape;
    int best_grid = b->grid;
    hipError_t e = hipSuccess;
    for (int w = 0; w < 3 && e == hipSuccess && s == LBK_OK; ++w) {
        for (int r = 0; r < 4 && e == hipSuccess && s == LBK_OK; ++r) {
            if ((s = set_shape(b, Shape{widths[w], row_opts[r]})) != LBK_OK)
                break;
            for (int c = 0; c < 4 && e == hipSuccess; ++c) {
                const int grid = per_cu[c] * b->cus;
                // every launch reads the current level and writes the other
                e = sweep_once(b, b->parity, grid, b->stream);
                if (e == hipSuccess)
                    e = hipEventRecord(ev[0], b->stream);
                for (int k = 0; k < reps && e == hipSuccess; ++k)
                    e = sweep_once(b, b->parity, grid, b->stream);
                if (e == hipSuccess)
                    e = hipEventRecord(ev[1], b->stream);
                if (e == hipSuccess)
                    e = hipEventSynchronize(ev[1]);
                float ms = 0.0f;
                if (e == hipSuccess)
                    e = hipEventElapsedTime(&ms, ev[0], ev[1]);
                if (e == hipSuccess && ms / reps < best) {
                    best = ms / reps;
                    best_shape = b->shape;
                    best_grid = grid;
                }
            }
        }
    }
    (void)hipEventDestroy(ev[0]);
    (void)hipEventDestroy(ev[1]);
    if (s != LBK_OK)
        return s;
    if (e != hipSuccess)
        return fail(LBK_ERR_DEVICE, "autotune: %s", hipGetErrorString(e));
    if ((s = lbk_batch_set_launch(b, best_shape.tile_x, best_shape.rows, best_grid,
                                  b->graph_steps)) != LBK_OK)
        return s;
    if (best_us)
        *best_us = best * 1e3;
    return LBK_OK;
}

lbk_status lbk_batch_apparent_permeability(lbk_batch *b, double *k_app)
{
    if (!b || !k_app)
        return fail(LBK_ERR_INVALID_ARG, "NULL argument");
    lbk_status s = sync_tables(b, false);
    if (s != LBK_OK)
        return s;
    const lbk_desc &d = b->d0();
    const int nt = (int)b->B.read_tiles;
    HIP_TRY(launch_batch_macro(d.storage, d.bc_x, d.bc_y, b->desc_read(), b->map_read(), nt,
                               b->parity, b->partials(), b->stream));
    HIP_TRY(launch_batch_finish(b->desc_read(), b->n, b->partials(), MAC_SLOTS, nt, b->results(),
                                b->stream));
    HIP_TRY(hipMemcpyAsync(b->host_res, b->results(), (size_t)b->n * MAC_SLOTS * sizeof(double),
                           hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    for (int i = 0; i < b->n; ++i)
        k_app[i] = k_app_of(b->lats[i], b->host_res + (size_t)i * MAC_SLOTS);
    return LBK_OK;
}

lbk_status lbk_batch_check(lbk_batch *b)
{
    if (!b)
        return fail(LBK_ERR_INVALID_ARG, "batch is NULL");
    for (int i = 0; i < b->n; ++i) {
        lbk_status s = check_state(b->lats[i]);
        if (s == LBK_ERR_NONFINITE)
            return fail(s, "non-finite value in sample %d after %lld steps", i,
                        (long long)b->lats[i]->t);
        if (s != LBK_OK)
            return s;
    }
    return sync_tables(b, false);
}

} // extern "C"
