// lbk_batch.hip -- host side of the ensemble calls in include/lbk.h: the
// tile list over every sample, the per-sample descriptor tables, graph
// recording of step runs and the launch-configuration tuner.  The kernels
// are the batched forms in lbk_kernels.hip.
#include "lbk_adjoint.h"
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

// Two-step pass tiling: groups of four 60-column strips (one workgroup) by
// bands of band2_of(storage) rows.
int groups_of(int nx) { return ((nx + kStrip2 - 1) / kStrip2 + kBlock / 64 - 1) / (kBlock / 64); }

int64_t tiles2_of(const lbk_lattice *l)
{
    const int band = band2_of(l->d.storage);
    return (int64_t)groups_of(l->d.nx) * ((l->d.ny + band - 1) / band);
}

int64_t total_tiles2(lbk_lattice *const *lats, int n)
{
    int64_t t = 0;
    for (int i = 0; i < n; ++i)
        t += tiles2_of(lats[i]);
    return t;
}

// Workspace regions: descriptor table and tile -> sample map of the sweep
// (sized for the finest allowed tiling), of the two-step pass and of the
// read-out; read-out partials [MAC_SLOTS][read tiles] and per-sample sums
// [n][MAC_SLOTS].
struct BatchLayout {
    size_t desc_sweep, map_sweep, desc_sweep2, map_sweep2, desc_read, map_read;
    int64_t max_sweep_tiles, sweep2_tiles, read_tiles;
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
    B.sweep2_tiles = total_tiles2(lats, n);
    B.read_tiles = total_tiles(lats, n, kReadShape);
    B.desc_sweep = take((size_t)n * sizeof(SampleDesc));
    B.map_sweep = take((size_t)B.max_sweep_tiles * sizeof(int));
    B.desc_sweep2 = take((size_t)n * sizeof(SampleDesc));
    B.map_sweep2 = take((size_t)B.sweep2_tiles * sizeof(int));
    B.desc_read = take((size_t)n * sizeof(SampleDesc));
    B.map_read = take((size_t)B.read_tiles * sizeof(int));
    B.partials = take((size_t)MAC_SLOTS * (size_t)B.read_tiles * sizeof(double));
    B.results = take((size_t)n * MAC_SLOTS * sizeof(double));
    B.total = o;
    return B;
}

// A batched gradient: the per-sample plans (same n, c1, c2 for every
// sample), each sample's slice of the workspace, and the descriptor table at
// the workspace's start.
struct BatchAdj {
    bool valid = false;
    int objective = 0;
    int64_t n = 0, c1 = 0, c2 = 0, k1 = 0, k2 = 0;
    int64_t keep = 0; // trailing segments whose inner checkpoints the forward keeps
    bool two_level = false;
    std::vector<AdjPlan> plans;
    std::vector<size_t> base;
    std::vector<int64_t> t0;
    std::vector<double> a1, a2;
    std::vector<int> outlet;
    size_t table = 0, total = 0;
    const void *ws = nullptr;
};

// Sample slices for `keep` kept segments (every sample keeps the same
// ones); returns the workspace total.
size_t batch_adj_place(BatchAdj &A, int64_t keep)
{
    const int n = (int)A.plans.size();
    // descriptor tables: the sweep's tiling, then the two-step tiling
    size_t o = align_up((size_t)2 * n * sizeof(AdjSampleDesc), 256);
    for (int i = 0; i < n; ++i) {
        AdjPlan &P = A.plans[i];
        P.total = P.inner + (size_t)(keep > 1 ? keep : 1) * P.inner_seg;
        P.keep = P.two_level ? keep : 0;
        A.base[i] = o;
        o = align_up(o + P.total, 256);
    }
    A.keep = A.two_level ? keep : 0;
    A.total = o;
    return o;
}

// Layout of a batched gradient; with ws_bytes beyond the minimum, the
// inner checkpoints of as many trailing segments as fit are kept.
lbk_status batch_adj_layout(lbk_lattice *const *lats, int n, int64_t steps, int64_t c1,
                            int64_t c2, BatchAdj &A, size_t ws_bytes = 0)
{
    A.plans.assign(n, AdjPlan{});
    A.base.assign(n, 0);
    A.table = 0;
    for (int i = 0; i < n; ++i) {
        lbk_status s = adj_plan(lats[i], steps, c1, c2, A.plans[i]);
        if (s != LBK_OK)
            return s;
    }
    A.n = steps;
    A.c1 = A.plans[0].c1;
    A.c2 = A.plans[0].c2;
    A.k1 = A.plans[0].k1;
    A.k2 = A.plans[0].k2;
    A.two_level = A.plans[0].two_level;
    int64_t keep = 1;
    if (A.two_level)
        for (int64_t K = A.k1; K > 1; --K)
            if (batch_adj_place(A, K) <= ws_bytes) {
                keep = K;
                break;
            }
    batch_adj_place(A, keep);
    return LBK_OK;
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
    std::vector<uint64_t> ver0; // each lattice's version when the tables were last set
    Shape shape;        // sweep tiling
    int64_t sweep_tiles;
    std::vector<int64_t> tile0_sweep, tile0_read, tile0_sweep2;
    int pass_mode;         // lbk_pass_mode asked for
    int tuned_two;         // -1: not tuned; else the tuner's choice (AUTO)
    SampleDesc *host_desc; // pinned staging, [3][n]: sweep, read-out, two-step pass
    double *host_res;      // pinned, [n][MAC_SLOTS]
    int grid, graph_steps;
    hipGraphExec_t exec[2]; // graphs starting at parity 0 / 1
    bool have_exec[2];
    bool graph_readout;     // graphs end with the per-sample read-out sums
    bool sums_fresh;        // results() holds the sums of the current state
    BatchAdj adj;           // the last batched gradient's forward pass

    SampleDesc *desc_sweep() const { return reinterpret_cast<SampleDesc *>(ws + B.desc_sweep); }
    SampleDesc *desc_sweep2() const { return reinterpret_cast<SampleDesc *>(ws + B.desc_sweep2); }
    int *map_sweep2() const { return reinterpret_cast<int *>(ws + B.map_sweep2); }
    SampleDesc *desc_read() const { return reinterpret_cast<SampleDesc *>(ws + B.desc_read); }
    int *map_sweep() const { return reinterpret_cast<int *>(ws + B.map_sweep); }
    int *map_read() const { return reinterpret_cast<int *>(ws + B.map_read); }
    double *partials() const { return reinterpret_cast<double *>(ws + B.partials); }
    double *results() const { return reinterpret_cast<double *>(ws + B.results); }
    const lbk_desc &d0() const { return lats[0]->d; }
    // whether steps go through the two-step pass (in pairs)
    bool two() const
    {
        if (pass_mode == LBK_PASS_TWO_STEP)
            return true;
        if (pass_mode == LBK_PASS_SINGLE)
            return false;
        if (tuned_two >= 0)
            return tuned_two != 0;
        int64_t nodes = 0;
        for (const lbk_lattice *l : lats)
            nodes += (int64_t)l->d.nx * l->d.ny;
        return nodes >= kTwoStepBatchNodes;
    }
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

// Upload the tile -> sample map of tiling `sh` (rows 0: the two-step
// pass's tiling) into `map`; tile0[i] gets the first tile of sample i.
// Synchronous.
lbk_status upload_map(lbk_batch *b, Shape sh, int *map, std::vector<int64_t> &tile0,
                      int64_t &ntiles)
{
    std::vector<int> h;
    tile0.assign(b->n, 0);
    for (int i = 0; i < b->n; ++i) {
        tile0[i] = (int64_t)h.size();
        h.insert(h.end(), (size_t)(sh.rows ? tiles_of(b->lats[i], sh) : tiles2_of(b->lats[i])), i);
    }
    ntiles = (int64_t)h.size();
    HIP_TRY(hipStreamSynchronize(b->stream));
    HIP_TRY(hipMemcpy(map, h.data(), h.size() * sizeof(int), hipMemcpyHostToDevice));
    return LBK_OK;
}

// Bring the device descriptor tables in line with the lattices: a lattice
// stepped, loaded or rescaled outside the batch changes its version (and may
// change which of its levels is current or its FP16 scale); then the tables
// are re-uploaded and the cached read-out sums dropped.
lbk_status sync_tables(lbk_batch *b, bool force)
{
    bool stale = force;
    for (int i = 0; i < b->n && !stale; ++i) {
        const lbk_lattice *l = b->lats[i];
        stale = l->cur != (b->cur0[i] ^ b->parity) || l->scale_exp != b->scale0[i] ||
                l->version != b->ver0[i];
    }
    if (!stale)
        return LBK_OK;
    b->sums_fresh = false;
    HIP_TRY(hipStreamSynchronize(b->stream)); // staging may still feed a copy
    for (int i = 0; i < b->n; ++i) {
        lbk_lattice *l = b->lats[i];
        b->cur0[i] = l->cur ^ b->parity;
        b->scale0[i] = l->scale_exp;
        b->ver0[i] = l->version;
        for (int k = 0; k < 3; ++k) {
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
            sd.tile0 = (int)(k == 0 ? b->tile0_sweep[i]
                                    : (k == 1 ? b->tile0_read[i] : b->tile0_sweep2[i]));
            sd.tpr = k == 2 ? groups_of(l->d.nx) : tiles_per_row(l->d.nx, sh.tile_x);
        }
    }
    HIP_TRY(hipMemcpyAsync(b->desc_sweep(), b->host_desc, (size_t)b->n * sizeof(SampleDesc),
                           hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipMemcpyAsync(b->desc_read(), b->host_desc + b->n, (size_t)b->n * sizeof(SampleDesc),
                           hipMemcpyHostToDevice, b->stream));
    HIP_TRY(hipMemcpyAsync(b->desc_sweep2(), b->host_desc + 2 * (size_t)b->n,
                           (size_t)b->n * sizeof(SampleDesc), hipMemcpyHostToDevice, b->stream));
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

// Two steps of every sample, parity -> parity ^ 1.
hipError_t sweep2_once(lbk_batch *b, int parity, hipStream_t st)
{
    const lbk_desc &d = b->d0();
    return launch_batch_sweep2(d.storage, d.bc_x, d.bc_y, b->desc_sweep2(), b->map_sweep2(),
                               (int)b->B.sweep2_tiles, parity, band2_of(d.storage), st);
}

// Per-sample read-out sums of the state at `parity` into results().
hipError_t readout(lbk_batch *b, int parity, hipStream_t st)
{
    const lbk_desc &d = b->d0();
    const int nt = (int)b->B.read_tiles;
    hipError_t e = launch_batch_macro(d.storage, d.bc_x, d.bc_y, b->desc_read(), b->map_read(),
                                      nt, parity, b->partials(), st);
    if (e == hipSuccess)
        e = launch_batch_finish(b->desc_read(), b->n, b->partials(), MAC_SLOTS, nt,
                                b->results(), st);
    return e;
}

// Parity after a graph replay of graph_steps steps from `parity`: single
// steps flip it each step (an even count), two-step passes once a pass.
int parity_after_graph(const lbk_batch *b, int parity)
{
    return b->two() ? parity ^ ((b->graph_steps / 2) & 1) : parity;
}

// Record graph_steps steps starting at `parity` on the private stream
// (and, with graph_readout, the read-out of the state they end in).
lbk_status record_graph(lbk_batch *b, int parity)
{
    HIP_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    if (b->two())
        for (int i = 0; i < b->graph_steps / 2 && e == hipSuccess; ++i)
            e = sweep2_once(b, parity ^ (i & 1), b->cap);
    else
        for (int i = 0; i < b->graph_steps && e == hipSuccess; ++i)
            e = sweep_once(b, parity ^ (i & 1), b->grid, b->cap);
    if (e == hipSuccess && b->graph_readout)
        e = readout(b, parity_after_graph(b, parity), b->cap);
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
    b->ver0.assign(n, 0);
    b->shape = Shape{0, 0};
    b->sweep_tiles = 0;
    b->grid = 0;
    b->graph_steps = 0;
    b->graph_readout = false;
    b->sums_fresh = false;
    int64_t read_tiles = 0;
    if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess ||
        hipHostMalloc((void **)&b->host_desc, (size_t)3 * n * sizeof(SampleDesc),
                      hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void **)&b->host_res, (size_t)n * MAC_SLOTS * sizeof(double),
                      hipHostMallocDefault) != hipSuccess) {
        destroy_batch(b);
        return fail(LBK_ERR_DEVICE, "stream or pinned host allocation failed");
    }
    b->pass_mode = LBK_PASS_AUTO;
    b->tuned_two = -1;
    int64_t sweep2_tiles = 0;
    if ((s = upload_map(b, kReadShape, b->map_read(), b->tile0_read, read_tiles)) != LBK_OK ||
        (s = upload_map(b, Shape{kStrip2, 0}, b->map_sweep2(), b->tile0_sweep2,
                        sweep2_tiles)) != LBK_OK ||
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
    const bool two = b->two();
    while (left > 0) {
        if (b->graph_steps > 0 && left >= b->graph_steps) {
            if (!b->have_exec[b->parity] && (s = record_graph(b, b->parity)) != LBK_OK)
                return s;
            Range range("batch graph replay");
            HIP_TRY(hipGraphLaunch(b->exec[b->parity], b->stream));
            left -= b->graph_steps;
            b->parity = parity_after_graph(b, b->parity);
            b->sums_fresh = b->graph_readout;
        } else if (two && left >= 2) {
            HIP_TRY(sweep2_once(b, b->parity, b->stream));
            b->parity ^= 1;
            left -= 2;
            b->sums_fresh = false;
        } else {
            HIP_TRY(sweep_once(b, b->parity, b->grid, b->stream));
            b->parity ^= 1;
            --left;
            b->sums_fresh = false;
        }
    }
    for (int i = 0; i < b->n; ++i) {
        lbk_lattice *l = b->lats[i];
        l->cur = b->cur0[i] ^ b->parity;
        l->t += n;
        if (n > 0)
            b->ver0[i] = ++l->version; // the batch's own change: tables stay valid
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

lbk_status lbk_batch_set_graph_readout(lbk_batch *b, int32_t on)
{
    if (!b)
        return fail(LBK_ERR_INVALID_ARG, "batch is NULL");
    if ((on != 0) != b->graph_readout)
        drop_graphs(b);
    b->graph_readout = on != 0;
    return LBK_OK;
}

lbk_status lbk_batch_set_pass_mode(lbk_batch *b, int32_t pass_mode)
{
    if (!b)
        return fail(LBK_ERR_INVALID_ARG, "batch is NULL");
    if (pass_mode < LBK_PASS_AUTO || pass_mode > LBK_PASS_SINGLE)
        return fail(LBK_ERR_INVALID_ARG, "pass_mode must be 0..2 (got %d)", pass_mode);
    const bool before = b->two();
    b->pass_mode = pass_mode;
    b->tuned_two = -1;
    if (b->two() != before)
        drop_graphs(b);
    return LBK_OK;
}

lbk_status lbk_batch_get_pass_mode(const lbk_batch *b, int32_t *pass_mode,
                                   int32_t *steps_per_launch)
{
    if (!b)
        return fail(LBK_ERR_INVALID_ARG, "batch is NULL");
    if (pass_mode)
        *pass_mode = b->pass_mode;
    if (steps_per_launch)
        *steps_per_launch = b->two() ? 2 : 1;
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
    // the two-step pass against the best single step, per step (automatic
    // pass mode only)
    int two = -1;
    if (s == LBK_OK && e == hipSuccess && b->pass_mode == LBK_PASS_AUTO) {
        e = sweep2_once(b, b->parity, b->stream);
        if (e == hipSuccess)
            e = hipEventRecord(ev[0], b->stream);
        for (int k = 0; k < reps && e == hipSuccess; ++k)
            e = sweep2_once(b, b->parity, b->stream);
        if (e == hipSuccess)
            e = hipEventRecord(ev[1], b->stream);
        if (e == hipSuccess)
            e = hipEventSynchronize(ev[1]);
        float ms = 0.0f;
        if (e == hipSuccess)
            e = hipEventElapsedTime(&ms, ev[0], ev[1]);
        if (e == hipSuccess) {
            two = ms / (2.0 * reps) < best ? 1 : 0;
            if (two)
                best = ms / (2.0 * reps);
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
    if (two >= 0 && two != b->tuned_two) {
        drop_graphs(b);
        b->tuned_two = two;
    }
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
    if (!b->sums_fresh) // else the last graph replay already reduced this state
        HIP_TRY(readout(b, b->parity, b->stream));
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

// ------------------------------------------------------------ gradients

namespace {

// Copy every sample's level `from` (ADJ_CUR: the lattice's current level)
// to level `to` of its adjoint workspace slice.
lbk_status copy_levels(lbk_batch *b, char *w, LevelSel from, LevelSel to)
{
    const BatchAdj &A = b->adj;
    for (int i = 0; i < b->n; ++i) {
        lbk_lattice *l = b->lats[i];
        const AdjPlan &P = A.plans[i];
        char *base = w + A.base[i];
        auto at = [&](LevelSel s) -> char * {
            if (s.region == ADJ_CUR)
                return l->state(l->cur);
            const size_t off = s.region == ADJ_OUTER ? P.outer
                               : s.region == ADJ_INNER ? P.inner : P.rec;
            return base + off + (size_t)s.index * P.level_bytes;
        };
        HIP_TRY(hipMemcpyAsync(at(to), at(from), P.level_bytes, hipMemcpyDeviceToDevice,
                               b->stream));
    }
    return LBK_OK;
}

} // namespace

extern "C" {

lbk_status lbk_batch_adjoint_workspace_size(lbk_batch *b, int64_t n_steps, int64_t ckpt_every,
                                            int64_t hist_len, size_t *bytes)
{
    if (!b || !bytes)
        return fail(LBK_ERR_INVALID_ARG, "NULL argument");
    BatchAdj A;
    lbk_status s = batch_adj_layout(b->lats.data(), b->n, n_steps, ckpt_every, hist_len, A);
    if (s != LBK_OK)
        return s;
    *bytes = A.total;
    return LBK_OK;
}

lbk_status lbk_batch_adjoint_plan(lbk_batch *b, int64_t n_steps, int64_t ckpt_every,
                                  size_t budget_bytes, int64_t *hist_len, size_t *bytes)
{
    if (!b || !hist_len)
        return fail(LBK_ERR_INVALID_ARG, "NULL argument");
    if (n_steps < 1 || ckpt_every < 1)
        return fail(LBK_ERR_INVALID_ARG, "need n_steps >= 1 and ckpt_every >= 1");
    const int64_t c1 = ckpt_every < n_steps ? ckpt_every : n_steps;
    // fewest sweeps rebuilding inner checkpoints; among equals, the longest
    // history
    int64_t prev = -1, best_h = -1, best_cost = -1;
    size_t best_bytes = 0;
    for (int64_t m = 1; m <= c1; ++m) {
        const int64_t h = (c1 + m - 1) / m;
        if (h == prev)
            continue;
        prev = h;
        BatchAdj A;
        lbk_status s = batch_adj_layout(b->lats.data(), b->n, n_steps, c1, h, A);
        if (s != LBK_OK)
            return s;
        if (A.total > budget_bytes)
            continue;
        if ((s = batch_adj_layout(b->lats.data(), b->n, n_steps, c1, h, A, budget_bytes)) !=
            LBK_OK)
            return s;
        const int64_t cost = adj_rebuild_steps(A.plans[0]);
        if (best_h < 0 || cost < best_cost) {
            best_h = h;
            best_cost = cost;
            best_bytes = A.total;
        }
        if (cost == 0)
            break;
    }
    if (best_h < 0)
        return fail(LBK_ERR_OOM, "no batched checkpoint plan fits in %zu bytes", budget_bytes);
    *hist_len = best_h;
    if (bytes)
        *bytes = best_bytes;
    return LBK_OK;
}

lbk_status lbk_batch_adjoint_forward(lbk_batch *b, int objective, int64_t n_steps,
                                     int64_t ckpt_every, int64_t hist_len, void *ws,
                                     size_t ws_bytes, double *J)
{
    if (!b || !ws || !J)
        return fail(LBK_ERR_INVALID_ARG, "NULL argument");
    if ((uintptr_t)ws & 255u)
        return fail(LBK_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    Range range("batch adjoint forward");
    for (int i = 0; i < b->n; ++i) {
        lbk_status s = check_objective(b->lats[i], objective);
        if (s != LBK_OK)
            return fail(s, "sample %d: %s", i, lbk_last_error());
    }
    BatchAdj &A = b->adj;
    A.valid = false;
    lbk_status s = batch_adj_layout(b->lats.data(), b->n, n_steps, ckpt_every, hist_len, A);
    if (s != LBK_OK)
        return s;
    if (ws_bytes < A.total)
        return fail(LBK_ERR_OOM, "batched adjoint workspace of %zu bytes < %zu needed", ws_bytes,
                    A.total);
    if ((s = batch_adj_layout(b->lats.data(), b->n, n_steps, ckpt_every, hist_len, A,
                              ws_bytes)) != LBK_OK)
        return s;
    if ((s = sync_tables(b, false)) != LBK_OK)
        return s;
    char *w = static_cast<char *>(ws);
    A.t0.assign(b->n, 0);
    for (int i = 0; i < b->n; ++i)
        A.t0[i] = b->lats[i]->t;
    for (int64_t k = 0; k < A.k1; ++k) {
        if ((s = copy_levels(b, w, LevelSel{ADJ_CUR, 0}, LevelSel{ADJ_OUTER, (int)k})) != LBK_OK)
            return s;
        const int64_t steps = std::min(A.c1, A.n - k * A.c1);
        const int64_t kept = k - (A.k1 - A.keep);
        if (A.two_level && kept >= 0) {
            // the last `keep` segments are reversed first: keep their inner
            // checkpoints
            for (int64_t i = 0; i < steps; i += A.c2) {
                if ((s = copy_levels(b, w, LevelSel{ADJ_CUR, 0},
                                     LevelSel{ADJ_INNER, (int)(kept * A.k2 + i / A.c2)})) !=
                        LBK_OK ||
                    (s = lbk_batch_step(b, std::min(A.c2, steps - i))) != LBK_OK)
                    return s;
            }
        } else if ((s = lbk_batch_step(b, steps)) != LBK_OK) {
            return s;
        }
    }
    // J of every sample from one batched read-out
    if (!b->sums_fresh)
        HIP_TRY(readout(b, b->parity, b->stream));
    HIP_TRY(hipMemcpyAsync(b->host_res, b->results(), (size_t)b->n * MAC_SLOTS * sizeof(double),
                           hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    A.a1.assign(b->n, 0.0);
    A.a2.assign(b->n, 0.0);
    A.outlet.assign(b->n, 0);
    for (int i = 0; i < b->n; ++i)
        J[i] = objective_weights(b->lats[i], objective, b->host_res + (size_t)i * MAC_SLOTS,
                                 A.a1[i], A.a2[i], A.outlet[i]);
    A.objective = objective;
    A.ws = ws;
    A.valid = true;
    return LBK_OK;
}

lbk_status lbk_batch_adjoint_backward(lbk_batch *b, void *ws, size_t ws_bytes,
                                      float *const *dJ_dlnk, float *const *dJ_dlnkn0)
{
    if (!b || !ws || !dJ_dlnk)
        return fail(LBK_ERR_INVALID_ARG, "NULL argument");
    BatchAdj &A = b->adj;
    if (!A.valid || A.ws != ws || ws_bytes < A.total)
        return fail(LBK_ERR_INVALID_ARG,
                    "no matching lbk_batch_adjoint_forward for this workspace");
    const bool kn = dJ_dlnkn0 != nullptr;
    for (int i = 0; i < b->n; ++i) {
        if (b->lats[i]->t != A.t0[i] + A.n)
            return fail(LBK_ERR_INVALID_ARG, "sample %d moved since the forward pass", i);
        if (!dJ_dlnk[i] || (kn && !dJ_dlnkn0[i]))
            return fail(LBK_ERR_INVALID_ARG, "output plane of sample %d is NULL", i);
    }
    char *w = static_cast<char *>(ws);
    hipStream_t st = b->stream;
    // descriptor tables of this pass: the sweep's tiling (one workgroup per
    // tile), then the same descriptors over the two-step tiling
    std::vector<AdjSampleDesc> h(2 * (size_t)b->n);
    for (int i = 0; i < b->n; ++i) {
        lbk_lattice *l = b->lats[i];
        const AdjPlan &P = A.plans[i];
        char *base = w + A.base[i];
        AdjSampleDesc &sd = h[i];
        sd.region[ADJ_CUR] = l->state(l->cur);
        sd.region[ADJ_OUTER] = base + P.outer;
        sd.region[ADJ_INNER] = base + P.inner;
        sd.region[ADJ_REC] = base + P.rec;
        sd.level_bytes = P.level_bytes;
        sd.hist = reinterpret_cast<float *>(base + P.hist);
        sd.hist_bytes = P.hist_bytes;
        sd.lam[0] = reinterpret_cast<float *>(base + P.lam);
        sd.lam[1] = reinterpret_cast<float *>(base + P.lam + P.lam_bytes);
        sd.seg = reinterpret_cast<float *>(base + P.seg);
        sd.seg2 = reinterpret_cast<float *>(base + P.seg2);
        sd.grad = reinterpret_cast<double *>(base + P.grad);
        sd.grad2 = reinterpret_cast<double *>(base + P.grad2);
        sd.out = dJ_dlnk[i];
        sd.out2 = kn ? dJ_dlnkn0[i] : nullptr;
        sd.med = l->med();
        sd.lay = l->L.lay;
        sd.mlay = l->L.mlay;
        sd.g = l->g;
        sd.ph = l->ph;
        sd.s = l->s();
        sd.inv_s = l->inv_s();
        sd.a1 = (float)A.a1[i];
        sd.a2 = (float)A.a2[i];
        sd.outlet = A.outlet[i];
        sd.tile0 = (int)b->tile0_sweep[i];
        sd.tpr = tiles_per_row(l->d.nx, b->shape.tile_x);
        AdjSampleDesc &s2 = h[(size_t)b->n + i];
        s2 = sd;
        s2.tile0 = (int)b->tile0_sweep2[i];
        s2.tpr = groups_of(l->d.nx);
    }
    AdjSampleDesc *table = reinterpret_cast<AdjSampleDesc *>(w + A.table);
    HIP_TRY(hipMemcpyAsync(table, h.data(), h.size() * sizeof(AdjSampleDesc),
                           hipMemcpyHostToDevice, st));
    const lbk_desc &d = b->d0();
    const int *map = b->map_sweep();
    const int nt = (int)b->sweep_tiles, tx = b->shape.tile_x, rows = b->shape.rows, knf = kn;
    auto rec = [&](LevelSel src, LevelSel dst, int slot) {
        return launch_batch_rec_sweep(d.storage, d.bc_x, d.bc_y, table, map, nt, tx, rows, src,
                                      dst, slot, st);
    };
    // pairs of steps through the two-step passes (bitwise the same) when
    // the batch steps that way
    const bool two = b->two();
    const AdjSampleDesc *table2 = table + b->n;
    const int nt2 = (int)b->B.sweep2_tiles, band = band2_of(d.storage);
    auto rec2 = [&](LevelSel src, LevelSel dst, int slot) {
        return launch_batch_rec_sweep2(d.storage, d.bc_x, d.bc_y, table2, b->map_sweep2(), nt2,
                                       band, src, dst, slot, st);
    };
    int fc = 0;
    for (int i = 0; i < b->n; ++i)
        fc |= b->lats[i]->d.f_eps != 0.0;
    auto reverse = [&](int lam_in, int slot) {
        return launch_batch_adjoint(d.bc_x, d.bc_y, table, map, nt, tx, rows, lam_in, slot, knf,
                                    fc, st);
    };
    auto reverse2 = [&](int lam_in, int slot) {
        return launch_batch_adjoint2(d.bc_x, d.bc_y, table2, b->map_sweep2(), nt2, band, lam_in,
                                     slot, knf, fc, st);
    };
    HIP_TRY(launch_batch_grad(table, map, nt, tx, rows, 0, knf, st));
    // read-out of J at step n: linearisation point of the pull of S_n
    HIP_TRY(rec(LevelSel{ADJ_CUR, 0}, LevelSel{ADJ_REC, 0}, 0));
    HIP_TRY(reverse(-1, 0));
    int cur = 0;
    for (int64_t k = A.k1 - 1; k >= 0; --k) {
        const int64_t a = k * A.c1, e = std::min(A.n, a + A.c1);
        int64_t nseg = 1;
        // inner checkpoints kept by the forward pass, or rebuilt into the
        // first kept segment's slots (free by now)
        const int64_t kept = k - (A.k1 - A.keep);
        const int i0 = (int)((kept > 0 ? kept : 0) * A.k2);
        if (A.two_level && kept >= 0) {
            nseg = (e - a + A.c2 - 1) / A.c2;
        } else if (A.two_level) {
            // rebuild the inner checkpoints of this outer segment
            Range range("batch adjoint rebuild");
            LevelSel src{ADJ_OUTER, (int)k};
            int r = 0;
            nseg = 0;
            for (int64_t t = a; t < e; t += A.c2, ++nseg) {
                lbk_status s = copy_levels(b, w, src, LevelSel{ADJ_INNER, (int)nseg});
                if (s != LBK_OK)
                    return s;
                const int64_t steps = std::min(A.c2, e - t);
                if (t + steps >= e)
                    break;
                for (int64_t i = 0; i < steps;) {
                    const LevelSel from =
                        i == 0 ? LevelSel{ADJ_INNER, (int)nseg} : LevelSel{ADJ_REC, r};
                    if (two && i + 1 < steps) {
                        HIP_TRY(rec2(from, LevelSel{ADJ_REC, r ^ 1}, -1));
                        i += 2;
                    } else {
                        HIP_TRY(rec(from, LevelSel{ADJ_REC, r ^ 1}, -1));
                        ++i;
                    }
                    r ^= 1;
                }
                src = LevelSel{ADJ_REC, r};
            }
            ++nseg;
        }
        for (int64_t j = nseg - 1; j >= 0; --j) {
            const int64_t a2s = A.two_level ? a + j * A.c2 : a;
            const int64_t b2s = A.two_level ? std::min(e, a2s + A.c2) : e;
            const LevelSel src = A.two_level ? LevelSel{ADJ_INNER, i0 + (int)j}
                                             : LevelSel{ADJ_OUTER, (int)k};
            int r = 0;
            {
                Range range("batch adjoint recompute");
                for (int64_t t = a2s; t < b2s;) {
                    const LevelSel from = t == a2s ? src : LevelSel{ADJ_REC, r};
                    if (two && t + 1 < b2s) {
                        HIP_TRY(rec2(from, LevelSel{ADJ_REC, r ^ 1}, (int)(t - a2s + 1)));
                        t += 2;
                    } else {
                        HIP_TRY(rec(from, LevelSel{ADJ_REC, r ^ 1}, (int)(t - a2s + 1)));
                        ++t;
                    }
                    r ^= 1;
                }
            }
            Range range("batch adjoint reverse");
            for (int64_t t = b2s; t > a2s;) {
                if (two && t - 1 > a2s) {
                    HIP_TRY(reverse2(cur, (int)(t - a2s)));
                    t -= 2;
                } else {
                    HIP_TRY(reverse(cur, (int)(t - a2s)));
                    --t;
                }
                cur ^= 1;
            }
            HIP_TRY(launch_batch_grad(table, map, nt, tx, rows, 1, knf, st));
        }
    }
    HIP_TRY(launch_batch_grad(table, map, nt, tx, rows, 2, knf, st));
    // the host copy of the table must outlive the upload
    HIP_TRY(hipStreamSynchronize(st));
    return LBK_OK;
}

} // extern "C"
