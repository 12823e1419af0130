// lbk3_api.hip -- host side of the D3Q19 calls of include/lbk.h: argument
// validation, workspace carve-up, launch sequencing and FP64 read-outs.
#include "lbk3_kernels.h"
#include "lbk_host.h"

#include <math.h>
#include <string.h>

#include <new>

using namespace lbk;

namespace {

// Workspace regions: two time levels of (ny nz) row blocks [rho | h_0..h_18]
// (pitch elements per slot), the medium row blocks [eps | drag | kn0], FP64
// partials and results.
struct WsLayout3 {
    int pitch;
    Layout lay;
    MLayout mlay;
    size_t level_bytes, level[2], med, partials, results, total;
    int blocks;
};

WsLayout3 layout3_of(const lbk_desc3 &d)
{
    WsLayout3 L{};
    L.pitch = (int)align_up((size_t)d.nx, 64);
    const size_t es = d.storage == LBK_F32 ? 4 : 2, p = (size_t)L.pitch;
    const size_t rows = (size_t)d.ny * d.nz;
    L.lay.row = p * (4 + 19 * es);
    L.lay.h_off = (uint32_t)(p * 4);
    L.lay.h_slot = (uint32_t)(p * es);
    L.mlay.row = 3 * p * 4;
    L.mlay.slot = (uint32_t)(p * 4);
    L.level_bytes = L.lay.row * rows;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes, 256);
        return at;
    };
    L.level[0] = take(L.level_bytes);
    L.level[1] = take(L.level_bytes);
    L.med = take(L.mlay.row * rows);
    L.blocks = blocks3_of(Geom3{d.nx, d.ny, d.nz, L.pitch});
    L.partials = take((size_t)8 * L.blocks * sizeof(double));
    L.results = take(8 * sizeof(double));
    L.total = o;
    return L;
}

lbk_status check_desc3(const lbk_desc3 *d)
{
    if (!d)
        return fail(LBK_ERR_INVALID_ARG, "desc is NULL");
    if (d->nx < 1 || d->ny < 1 || d->nz < 1)
        return fail(LBK_ERR_INVALID_ARG, "nx, ny, nz must be >= 1");
    if ((int64_t)align_up((size_t)d->nx, 64) * d->ny * d->nz > (int64_t)1 << 30 ||
        (int64_t)d->ny * d->nz > (int64_t)1 << 24)
        return fail(LBK_ERR_UNSUPPORTED, "lattice of %d x %d x %d is too large", d->nx, d->ny,
                    d->nz);
    // row blocks are reached through buffer resources with 32-bit offsets;
    // the widest (an FP32 state row, 80 B per node) must fit
    if ((uint64_t)align_up((size_t)d->nx, 64) * 80 > 0xFFFFFFFFull)
        return fail(LBK_ERR_UNSUPPORTED, "rows of %d nodes exceed the 4 GiB a row block may span",
                    d->nx);
    if (d->bc_x < 0 || d->bc_x > 2 || d->bc_y < 0 || d->bc_y > 1 || d->bc_z < 0 || d->bc_z > 1)
        return fail(LBK_ERR_INVALID_ARG, "bc_x must be 0..2, bc_y and bc_z 0..1");
    if (d->storage < 0 || d->storage > 2)
        return fail(LBK_ERR_INVALID_ARG, "storage must be 0..2");
    if (!(d->tau > 0.5) || !isfinite(d->tau))
        return fail(LBK_ERR_INVALID_ARG, "tau must be > 1/2");
    if (!isfinite(d->gx) || !isfinite(d->gy) || !isfinite(d->gz) || !isfinite(d->f_eps) ||
        d->f_eps < 0)
        return fail(LBK_ERR_INVALID_ARG, "gx, gy, gz, f_eps must be finite, f_eps >= 0");
    if (d->bc_x == LBK_BC_PRESSURE && d->nx < 3)
        return fail(LBK_ERR_INVALID_ARG, "pressure boundaries need nx >= 3");
    if ((d->bc_x == LBK_BC_PRESSURE || d->init == 1) &&
        (!(d->rho_in > 0) || !(d->rho_out > 0) || !isfinite(d->rho_in) || !isfinite(d->rho_out)))
        return fail(LBK_ERR_INVALID_ARG, "rho_in, rho_out must be positive and finite");
    if (d->init != 0 && d->init != 1)
        return fail(LBK_ERR_INVALID_ARG, "init must be 0 or 1");
    if (d->init == 0 && (!(d->rho0 > 0) || !isfinite(d->rho0)))
        return fail(LBK_ERR_INVALID_ARG, "rho0 must be positive and finite");
    if (!(d->rho_ref > 0) || !isfinite(d->rho_ref))
        return fail(LBK_ERR_INVALID_ARG, "rho_ref must be positive and finite");
    if (d->check_every < 0)
        return fail(LBK_ERR_INVALID_ARG, "check_every must be >= 0");
    if (d->correlation < 0 || d->correlation > 2)
        return fail(LBK_ERR_INVALID_ARG, "correlation must be 0..2");
    if (!(d->slip_b <= 0.0) || !isfinite(d->slip_b))
        return fail(LBK_ERR_INVALID_ARG, "slip_b must be finite and <= 0");
    if (d->reserved != 0)
        return fail(LBK_ERR_INVALID_ARG, "reserved must be 0");
    return LBK_OK;
}

void split3(double v, float &hi, float &lo)
{
    hi = (float)v;
    lo = (float)(v - (double)hi);
}

} // namespace

struct lbk_lattice3 {
    lbk_desc3 d;
    WsLayout3 L;
    Geom3 g;
    Physics3 p3;
    hipStream_t stream;
    char *ws;
    int cur;
    int64_t t;
    int scale_exp;
    double eps_b;
    double *host;

    char *state(int l) const { return ws + L.level[l]; }
    char *med() const { return ws + L.med; }
    float s() const { return ldexpf(1.0f, scale_exp); }
    float inv_s() const { return ldexpf(1.0f, -scale_exp); }
    double *partials() const { return reinterpret_cast<double *>(ws + L.partials); }
    double *results() const { return reinterpret_cast<double *>(ws + L.results); }
};

namespace {

lbk_status fetch3(lbk_lattice3 *lat, int slots, unsigned max_mask)
{
    HIP_TRY(launch_finish(lat->partials(), slots, lat->L.blocks, max_mask, lat->results(),
                          lat->stream));
    HIP_TRY(hipMemcpyAsync(lat->host, lat->results(), slots * sizeof(double),
                           hipMemcpyDeviceToHost, lat->stream));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    return LBK_OK;
}

lbk_status check_state3(lbk_lattice3 *lat)
{
    HIP_TRY(launch_state_sums3(lat->d.storage, lat->state(lat->cur), lat->L.lay, lat->g,
                               lat->inv_s(), lat->partials(), lat->stream));
    lbk_status st = fetch3(lat, ST_SLOTS, 1u << ST_HMAX);
    if (st != LBK_OK)
        return st;
    if (lat->host[ST_BAD] != 0.0 || !isfinite(lat->host[ST_MASS]))
        return fail(LBK_ERR_NONFINITE, "non-finite value in the state after %lld steps",
                    (long long)lat->t);
    if (lat->d.storage == LBK_F16 && lat->host[ST_HMAX] > 0.0) {
        int e;
        frexp(lat->host[ST_HMAX] * ldexp(1.0, lat->scale_exp), &e);
        if (e > 14 || e < 10) {
            int k = 13 - e;
            if (lat->scale_exp + k > 100)
                k = 100 - lat->scale_exp;
            if (k != 0) {
                HIP_TRY(launch_rescale3(lat->d.storage, lat->state(lat->cur), lat->L.lay, lat->g,
                                        k, lat->stream));
                lat->scale_exp += k;
            }
        }
    }
    return LBK_OK;
}

} // namespace

extern "C" {

lbk_status lbk3_desc_default(lbk_desc3 *d)
{
    if (!d)
        return fail(LBK_ERR_INVALID_ARG, "desc is NULL");
    memset(d, 0, sizeof *d);
    d->nx = d->ny = d->nz = 1;
    d->storage = LBK_F32;
    d->kn_local = 1;
    d->check_every = 100;
    d->tau = 0.8;
    d->rho_in = d->rho_out = d->rho0 = d->rho_ref = 1.0;
    d->slip_b = -1.0;
    d->correlation = LBK_FC_BKC;
    return LBK_OK;
}

lbk_status lbk3_workspace_size(const lbk_desc3 *d, size_t *bytes)
{
    lbk_status s = check_desc3(d);
    if (s != LBK_OK)
        return s;
    if (!bytes)
        return fail(LBK_ERR_INVALID_ARG, "bytes is NULL");
    *bytes = layout3_of(*d).total;
    return LBK_OK;
}

lbk_status lbk3_create(const lbk_desc3 *d, const float *eps, const float *k, const float *kn0,
                       void *workspace, size_t ws_bytes, void *stream, lbk_lattice3 **out)
{
    if (!out)
        return fail(LBK_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    lbk_status s = check_desc3(d);
    if (s != LBK_OK)
        return s;
    if (!eps || !k)
        return fail(LBK_ERR_INVALID_ARG, "eps and k are required");
    if (!workspace || ((uintptr_t)workspace & 255u))
        return fail(LBK_ERR_INVALID_ARG, "workspace must be non-NULL and 256-byte aligned");
    const WsLayout3 L = layout3_of(*d);
    if (ws_bytes < L.total)
        return fail(LBK_ERR_OOM, "workspace of %zu bytes < %zu needed", ws_bytes, L.total);
    int dev = -1;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return fail(LBK_ERR_DEVICE, "no HIP device");
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(LBK_ERR_DEVICE, "device %s is not gfx950", prop.gcnArchName);
    lbk_lattice3 *lat = new (std::nothrow) lbk_lattice3();
    if (!lat)
        return fail(LBK_ERR_OOM, "host allocation failed");
    lat->d = *d;
    lat->L = L;
    lat->g = Geom3{d->nx, d->ny, d->nz, L.pitch};
    lat->stream = static_cast<hipStream_t>(stream);
    lat->ws = static_cast<char *>(workspace);
    lat->cur = 0;
    lat->t = 0;
    lat->scale_exp = d->storage == LBK_F16 ? 20 : 0;
    if (hipHostMalloc((void **)&lat->host, 8 * sizeof(double), hipHostMallocDefault) !=
        hipSuccess) {
        delete lat;
        return fail(LBK_ERR_DEVICE, "pinned host allocation failed");
    }
    auto cleanup = [&](lbk_status st) {
        (void)hipHostFree(lat->host);
        delete lat;
        return st;
    };
    const double nu = (d->tau - 0.5) / 3.0;
    Physics &ph = lat->p3.ph;
    ph.omega = (float)(1.0 / d->tau);
    ph.guo = (float)(1.0 - 0.5 / d->tau);
    ph.gx = (float)d->gx;
    ph.gy = (float)d->gy;
    lat->p3.gz = (float)d->gz;
    ph.feps = (float)d->f_eps;
    ph.inv_nu = (float)(1.0 / nu);
    ph.rho_ref = (float)d->rho_ref;
    split3(d->rho_in, ph.rin_hi, ph.rin_lo);
    split3(d->rho_out, ph.rout_hi, ph.rout_lo);
    ph.kn_local = d->kn_local ? 1 : 0;
    ph.corr = d->correlation;
    ph.slip_nb = (float)(-d->slip_b);
    ph.slip_c = (float)(4.0 - d->slip_b);

    hipStream_t st = lat->stream;
    char *med = lat->med();
    const size_t row = (size_t)d->nx * sizeof(float), rows = (size_t)d->ny * d->nz;
    const size_t mrow = L.mlay.row;
    auto ok = [&](hipError_t e, const char *what) {
        if (e == hipSuccess)
            return true;
        fail(LBK_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
        return false;
    };
    if (!ok(hipMemsetAsync(lat->ws, 0, L.total, st), "clear workspace") ||
        !ok(hipMemcpy2DAsync(med, mrow, eps, row, row, rows, hipMemcpyDefault, st), "eps") ||
        !ok(hipMemcpy2DAsync(med + L.mlay.slot, mrow, k, row, row, rows, hipMemcpyDefault, st),
            "k") ||
        (kn0 && !ok(hipMemcpy2DAsync(med + 2 * L.mlay.slot, mrow, kn0, row, row, rows,
                                     hipMemcpyDefault, st), "kn0")) ||
        !ok(launch_fields3(med, L.mlay, lat->g, nu, lat->partials(), st), "fields kernel"))
        return cleanup(LBK_ERR_DEVICE);
    if ((s = fetch3(lat, FLD_SLOTS, 0)) != LBK_OK)
        return cleanup(s);
    if (lat->host[FLD_BAD] != 0.0)
        return cleanup(fail(LBK_ERR_INVALID_ARG,
                            "%.0f field values out of range (need 0<=eps<=1, k>0 or +inf, "
                            "kn0>=0 finite)", lat->host[FLD_BAD]));
    lat->eps_b = 0.0;
    if (d->bc_x == LBK_BC_PRESSURE) {
        float *col = nullptr;
        if (hipHostMalloc((void **)&col, 2 * rows * sizeof(float), hipHostMallocDefault) !=
            hipSuccess)
            return cleanup(fail(LBK_ERR_DEVICE, "pinned host allocation failed"));
        bool good = ok(hipMemcpy2DAsync(col, sizeof(float), med, mrow, sizeof(float), rows,
                                        hipMemcpyDeviceToHost, st), "eps plane") &&
                    ok(hipMemcpy2DAsync(col + rows, sizeof(float),
                                        med + (d->nx - 1) * sizeof(float), mrow, sizeof(float),
                                        rows, hipMemcpyDeviceToHost, st), "eps plane") &&
                    ok(hipStreamSynchronize(st), "sync");
        double sum = 0.0;
        for (size_t i = 0; good && i < 2 * rows; ++i)
            sum += col[i];
        (void)hipHostFree(col);
        if (!good)
            return cleanup(LBK_ERR_DEVICE);
        lat->eps_b = sum / (2.0 * rows);
    }
    if (!ok(launch_init3(d->storage, lat->state(0), L.lay, lat->g, d->init, d->rho0, d->rho_in,
                         d->rho_out, lat->s(), st), "init kernel") ||
        !ok(hipStreamSynchronize(st), "sync"))
        return cleanup(LBK_ERR_DEVICE);
    *out = lat;
    return LBK_OK;
}

lbk_status lbk3_destroy(lbk_lattice3 *lat)
{
    if (!lat)
        return LBK_OK;
    (void)hipHostFree(lat->host);
    delete lat;
    return LBK_OK;
}

lbk_status lbk3_step(lbk_lattice3 *lat, int64_t n)
{
    if (!lat)
        return fail(LBK_ERR_INVALID_ARG, "lattice is NULL");
    if (n < 0)
        return fail(LBK_ERR_INVALID_ARG, "n must be >= 0");
    const lbk_desc3 &d = lat->d;
    Range range("lbk3_step");
    for (int64_t i = 0; i < n; ++i) {
        const int nxt = lat->cur ^ 1;
        HIP_TRY(launch_sweep3(d.storage, d.bc_x, d.bc_y, d.bc_z, lat->state(lat->cur),
                              lat->state(nxt), lat->L.lay, lat->med(), lat->L.mlay, lat->g,
                              lat->p3, lat->s(), lat->inv_s(), lat->stream));
        lat->cur = nxt;
        ++lat->t;
        // checks fall on multiples of check_every in the lattice's own time,
        // so a run resumed from a saved state checks where the original did
        if (d.check_every > 0 && lat->t % d.check_every == 0) {
            lbk_status s = check_state3(lat);
            if (s != LBK_OK)
                return s;
        }
    }
    return LBK_OK;
}

lbk_status lbk3_time(const lbk_lattice3 *lat, int64_t *t)
{
    if (!lat || !t)
        return fail(LBK_ERR_INVALID_ARG, "NULL argument");
    *t = lat->t;
    return LBK_OK;
}

lbk_status lbk3_scale_exponent(const lbk_lattice3 *lat, int32_t *e)
{
    if (!lat || !e)
        return fail(LBK_ERR_INVALID_ARG, "NULL argument");
    *e = lat->scale_exp;
    return LBK_OK;
}

lbk_status lbk3_read_macroscopic(lbk_lattice3 *lat, float *rho, float *ux, float *uy, float *uz)
{
    if (!lat)
        return fail(LBK_ERR_INVALID_ARG, "lattice is NULL");
    const lbk_desc3 &d = lat->d;
    HIP_TRY(launch_macro3(d.storage, d.bc_x, d.bc_y, d.bc_z, lat->state(lat->cur), lat->L.lay,
                          lat->med(), lat->L.mlay, lat->g, lat->p3, lat->s(), lat->inv_s(), rho,
                          ux, uy, uz, lat->partials(), lat->stream));
    return LBK_OK;
}

lbk_status lbk3_read_populations(lbk_lattice3 *lat, double *f)
{
    if (!lat || !f)
        return fail(LBK_ERR_INVALID_ARG, "NULL argument");
    HIP_TRY(launch_populations3(lat->d.storage, lat->state(lat->cur), lat->L.lay, lat->g,
                                lat->inv_s(), f, lat->stream));
    return LBK_OK;
}

lbk_status lbk3_apparent_permeability(lbk_lattice3 *lat, double *k_app)
{
    if (!lat || !k_app)
        return fail(LBK_ERR_INVALID_ARG, "NULL argument");
    if (lat->d.bc_x == LBK_BC_PRESSURE ? lat->d.rho_in == lat->d.rho_out : lat->d.gx == 0.0)
        return fail(LBK_ERR_INVALID_ARG, "the global permeability needs rho_in != rho_out "
                                         "(pressure drive) or gx != 0");
    lbk_status s = lbk3_read_macroscopic(lat, nullptr, nullptr, nullptr, nullptr);
    if (s != LBK_OK || (s = fetch3(lat, MAC_SLOTS, 0)) != LBK_OK)
        return s;
    const lbk_desc3 &d = lat->d;
    const double n = (double)d.nx * d.ny * d.nz, nu = (d.tau - 0.5) / 3.0;
    if (d.bc_x == LBK_BC_PRESSURE)
        *k_app = lat->eps_b * nu * (d.nx - 1) * (lat->host[MAC_FLUX] / n) /
                 ((1.0 / 3.0) * (d.rho_in - d.rho_out));
    else
        *k_app = nu * (lat->host[MAC_UX] / n) / d.gx;
    return LBK_OK;
}

lbk_status lbk3_diagnostics(lbk_lattice3 *lat, double *mass, double *flux_x)
{
    if (!lat)
        return fail(LBK_ERR_INVALID_ARG, "lattice is NULL");
    lbk_status s;
    if (flux_x) {
        if ((s = lbk3_read_macroscopic(lat, nullptr, nullptr, nullptr, nullptr)) != LBK_OK ||
            (s = fetch3(lat, MAC_SLOTS, 0)) != LBK_OK)
            return s;
        *flux_x = lat->host[MAC_FLUX];
    }
    if (mass) {
        HIP_TRY(launch_state_sums3(lat->d.storage, lat->state(lat->cur), lat->L.lay, lat->g,
                                   lat->inv_s(), lat->partials(), lat->stream));
        if ((s = fetch3(lat, ST_SLOTS, 1u << ST_HMAX)) != LBK_OK)
            return s;
        *mass = lat->host[ST_MASS];
    }
    return LBK_OK;
}

} // extern "C"
