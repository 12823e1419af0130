// lbk_api.hip -- host side of the C ABI declared in include/lbk.h: argument
// validation, workspace carve-up, launch sequencing on the caller's stream,
// FP64 diagnostics and state save/load.  No kernels live here.
#include "lbk_adjoint.h"
#include "lbk_host.h"

#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <new>
#include <string>

using namespace lbk;

namespace {
thread_local std::string g_err;
} // namespace

lbk_status lbk::fail(lbk_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

namespace {

size_t elem_size(int storage) { return storage == LBK_F32 ? 4 : 2; }

WsLayout layout_of(const lbk_desc &d)
{
    WsLayout L{};
    L.pitch = (int)align_up((size_t)d.nx, 64);
    const size_t es = elem_size(d.storage), p = (size_t)L.pitch;
    L.lay.row = p * (4 + 9 * es);
    L.lay.h_off = (uint32_t)(p * 4);
    L.lay.h_slot = (uint32_t)(p * es);
    L.mlay.row = 3 * p * 4;
    L.mlay.slot = (uint32_t)(p * 4);
    L.level_bytes = L.lay.row * (size_t)d.ny;
    const size_t f32 = p * (size_t)d.ny * 4;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes, 256);
        return at;
    };
    L.level[0] = take(L.level_bytes);
    L.level[1] = take(L.level_bytes);
    L.med = take(L.mlay.row * (size_t)d.ny);
    L.uxp = take(f32);
    L.uyp = take(f32);
    Geom g{d.nx, d.ny, L.pitch};
    L.blocks = launch_of(g).blocks;
    L.partials = take((size_t)8 * L.blocks * sizeof(double));
    L.results = take(8 * sizeof(double));
    L.total = o;
    return L;
}

lbk_status check_desc(const lbk_desc *d)
{
    if (!d)
        return fail(LBK_ERR_INVALID_ARG, "desc is NULL");
    if (d->nx < 1 || d->ny < 1)
        return fail(LBK_ERR_INVALID_ARG, "nx, ny must be >= 1 (got %d, %d)", d->nx, d->ny);
    if ((int64_t)align_up((size_t)d->nx, 64) * d->ny > (int64_t)1 << 30)
        return fail(LBK_ERR_UNSUPPORTED, "lattice of %d x %d exceeds 2^30 nodes", d->nx, d->ny);
    // kernels reach every row block through a buffer resource with 32-bit
    // offsets; the widest row (an FP32 state row, 40 B per node) must fit
    if ((uint64_t)align_up((size_t)d->nx, 64) * 40 > 0xFFFFFFFFull)
        return fail(LBK_ERR_UNSUPPORTED, "rows of %d nodes exceed the 4 GiB a row block may span",
                    d->nx);
    if (d->bc_x < 0 || d->bc_x > 2 || d->bc_y < 0 || d->bc_y > 1)
        return fail(LBK_ERR_INVALID_ARG, "bc_x must be 0..2 and bc_y 0..1 (got %d, %d)",
                    d->bc_x, d->bc_y);
    if (d->storage < 0 || d->storage > 2)
        return fail(LBK_ERR_INVALID_ARG, "storage must be 0..2 (got %d)", d->storage);
    if (!(d->tau > 0.5) || !isfinite(d->tau))
        return fail(LBK_ERR_INVALID_ARG, "tau must be > 1/2 (got %g)", d->tau);
    if (!isfinite(d->gx) || !isfinite(d->gy) || !isfinite(d->f_eps) || d->f_eps < 0)
        return fail(LBK_ERR_INVALID_ARG, "gx, gy, f_eps must be finite, f_eps >= 0");
    if (d->bc_x == LBK_BC_PRESSURE) {
        if (d->nx < 3)
            return fail(LBK_ERR_INVALID_ARG, "pressure boundaries need nx >= 3");
    }
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
        return fail(LBK_ERR_INVALID_ARG, "correlation must be 0..2 (got %d)", d->correlation);
    if (!(d->slip_b <= 0.0) || !isfinite(d->slip_b))
        return fail(LBK_ERR_INVALID_ARG, "slip_b must be finite and <= 0 (got %g)", d->slip_b);
    if (d->pass_mode < LBK_PASS_AUTO || d->pass_mode > LBK_PASS_THREE_STEP)
        return fail(LBK_ERR_INVALID_ARG, "pass_mode must be 0..3 (got %d)", d->pass_mode);
    if (d->band < 0 || d->band > 1024)
        return fail(LBK_ERR_INVALID_ARG, "band must be 0..1024 (got %d)", d->band);
    return LBK_OK;
}

// Split a double into hi + lo floats with hi + lo == v to ~2^-48 relative.
void split(double v, float &hi, float &lo)
{
    hi = (float)v;
    lo = (float)(v - (double)hi);
}

} // namespace

// n steps of the lattice on stream st: when the lattice takes three-step
// passes, triples of steps fused into one pass (launch_sweep3x), the rest
// in a two-step pass or a single sweep; when it takes two-step passes,
// pairs of steps fused into one pass (launch_sweep2) and a single sweep if
// n is odd; otherwise n single sweeps.  Every pass is bitwise the single
// sweeps it replaces.
lbk_status lbk::advance(lbk_lattice *lat, int64_t n, hipStream_t st)
{
    const lbk_desc &d = lat->d;
    int64_t i = 0;
    for (; three_step_pass(lat) && i + 2 < n; i += 3) {
        const int nxt = lat->cur ^ 1;
        HIP_TRY(launch_sweep3x(d.storage, d.bc_x, d.bc_y, lat->state(lat->cur),
                               lat->state(nxt), lat->L.lay, lat->med(), lat->L.mlay, lat->g,
                               lat->ph, lat->s(), lat->inv_s(), fwd_band3(d), nullptr,
                               nullptr, nullptr, st));
        lat->cur = nxt;
        lat->t += 3;
        ++lat->version;
    }
    for (; two_step_pass(lat) && i + 1 < n; i += 2) {
        const int nxt = lat->cur ^ 1;
        HIP_TRY(launch_sweep2(d.storage, d.bc_x, d.bc_y, lat->state(lat->cur), lat->state(nxt),
                              lat->L.lay, lat->med(), lat->L.mlay, lat->g, lat->ph, lat->s(),
                              lat->inv_s(), fwd_band(d), nullptr, nullptr, st));
        lat->cur = nxt;
        lat->t += 2;
        ++lat->version;
    }
    for (; i < n; ++i) {
        const int nxt = lat->cur ^ 1;
        HIP_TRY(launch_sweep(d.storage, d.bc_x, d.bc_y, lat->state(lat->cur), lat->state(nxt),
                             lat->L.lay, lat->med(), lat->L.mlay, lat->g, lat->ph, lat->s(),
                             lat->inv_s(), nullptr, st));
        lat->cur = nxt;
        ++lat->t;
        ++lat->version;
    }
    return LBK_OK;
}

// Run a reduction's finish kernel and copy `slots` doubles to lat->host.
lbk_status lbk::fetch(lbk_lattice *lat, int slots, unsigned max_mask)
{
    HIP_TRY(launch_finish(lat->partials(), slots, lat->L.blocks, max_mask, lat->results(),
                          lat->stream));
    HIP_TRY(hipMemcpyAsync(lat->host, lat->results(), slots * sizeof(double),
                           hipMemcpyDeviceToHost, lat->stream));
    HIP_TRY(hipStreamSynchronize(lat->stream));
    return LBK_OK;
}

// NaN/Inf check of the current state; for FP16 also re-centre the scale so
// the largest stored magnitude sits near 2^12 (exact power-of-two rescale).
lbk_status lbk::check_state(lbk_lattice *lat)
{
    char *s = lat->state(lat->cur);
    HIP_TRY(launch_state_sums(lat->d.storage, s, lat->L.lay, lat->g, lat->inv_s(),
                              lat->partials(), lat->stream));
    lbk_status st = fetch(lat, ST_SLOTS, 1u << ST_HMAX);
    if (st != LBK_OK)
        return st;
    if (lat->host[ST_BAD] != 0.0 || !isfinite(lat->host[ST_MASS]))
        return fail(LBK_ERR_NONFINITE, "non-finite value in the state after %lld steps",
                    (long long)lat->t);
    if (lat->d.storage == LBK_F16 && lat->host[ST_HMAX] > 0.0) {
        int e;
        frexp(lat->host[ST_HMAX] * ldexp(1.0, lat->scale_exp), &e); // stored max in [2^(e-1), 2^e)
        const int target = 13;                                       // max in [2^12, 2^13)
        if (e > 14 || e < 10) {
            int k = target - e;
            if (lat->scale_exp + k > 100)
                k = 100 - lat->scale_exp;
            if (k != 0) {
                HIP_TRY(launch_rescale(lat->d.storage, s, lat->L.lay, lat->g, k, lat->stream));
                lat->scale_exp += k;
                ++lat->version;
            }
        }
    }
    return LBK_OK;
}

extern "C" {

lbk_status lbk_desc_default(lbk_desc *d)
{
    if (!d)
        return fail(LBK_ERR_INVALID_ARG, "desc is NULL");
    memset(d, 0, sizeof *d);
    d->nx = d->ny = 1;
    d->bc_x = d->bc_y = LBK_BC_PERIODIC;
    d->storage = LBK_F32;
    d->kn_local = 1;
    d->init = 0;
    d->check_every = 100;
    d->tau = 0.8;
    d->rho_in = d->rho_out = d->rho0 = d->rho_ref = 1.0;
    d->slip_b = -1.0;
    d->correlation = LBK_FC_BKC;
    return LBK_OK;
}

lbk_status lbk_workspace_size(const lbk_desc *d, size_t *bytes)
{
    lbk_status s = check_desc(d);
    if (s != LBK_OK)
        return s;
    if (!bytes)
        return fail(LBK_ERR_INVALID_ARG, "bytes is NULL");
    *bytes = layout_of(*d).total;
    return LBK_OK;
}

lbk_status lbk_create(const lbk_desc *d, const float *eps, const float *k, const float *kn0,
                      void *workspace, size_t ws_bytes, void *stream, lbk_lattice **out)
{
    if (!out)
        return fail(LBK_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    lbk_status s = check_desc(d);
    if (s != LBK_OK)
        return s;
    if (!eps || !k)
        return fail(LBK_ERR_INVALID_ARG, "eps and k are required");
    if (!workspace || ((uintptr_t)workspace & 255u))
        return fail(LBK_ERR_INVALID_ARG, "workspace must be non-NULL and 256-byte aligned");
    WsLayout L = layout_of(*d);
    if (ws_bytes < L.total)
        return fail(LBK_ERR_OOM, "workspace of %zu bytes < %zu needed", ws_bytes, L.total);
    int dev = -1;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
        return fail(LBK_ERR_DEVICE, "no HIP device");
    if (strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(LBK_ERR_DEVICE, "device %s is not gfx950", prop.gcnArchName);

    lbk_lattice *lat = new (std::nothrow) lbk_lattice();
    if (!lat)
        return fail(LBK_ERR_OOM, "host allocation failed");
    lat->d = *d;
    lat->L = L;
    lat->g = Geom{d->nx, d->ny, L.pitch};
    lat->stream = static_cast<hipStream_t>(stream);
    lat->device = dev;
    lat->ws = static_cast<char *>(workspace);
    lat->cur = 0;
    lat->t = 0;
    lat->version = 0;
    lat->scale_exp = d->storage == LBK_F16 ? 20 : 0;
    lat->have_prev = false;
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
    Physics &ph = lat->ph;
    ph.omega = (float)(1.0 / d->tau);
    ph.guo = (float)(1.0 - 0.5 / d->tau);
    ph.gx = (float)d->gx;
    ph.gy = (float)d->gy;
    ph.feps = (float)d->f_eps;
    ph.inv_nu = (float)(1.0 / nu);
    ph.rho_ref = (float)d->rho_ref;
    split(d->rho_in, ph.rin_hi, ph.rin_lo);
    split(d->rho_out, ph.rout_hi, ph.rout_lo);
    ph.kn_local = d->kn_local ? 1 : 0;
    ph.corr = d->correlation;
    ph.slip_nb = (float)(-d->slip_b);
    ph.slip_c = (float)(4.0 - d->slip_b);

    char *ws = lat->ws;
    char *med = lat->med();
    const size_t row = (size_t)d->nx * sizeof(float), mrow = L.mlay.row;
    hipStream_t st = lat->stream;
    auto hip_ok = [&](hipError_t e, const char *what) {
        if (e == hipSuccess)
            return true;
        fail(LBK_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
        return false;
    };
    // raw fields into the medium slots (eps, k, kn0), then k -> drag
    if (!hip_ok(hipMemsetAsync(ws, 0, L.total, st), "clear workspace") ||
        !hip_ok(hipMemcpy2DAsync(med, mrow, eps, row, row, d->ny, hipMemcpyDefault, st), "eps") ||
        !hip_ok(hipMemcpy2DAsync(med + L.mlay.slot, mrow, k, row, row, d->ny, hipMemcpyDefault,
                                 st), "k") ||
        (kn0 && !hip_ok(hipMemcpy2DAsync(med + 2 * L.mlay.slot, mrow, kn0, row, row, d->ny,
                                         hipMemcpyDefault, st), "kn0")) ||
        !hip_ok(launch_fields(med, L.mlay, lat->g, nu, lat->partials(), st), "fields kernel"))
        return cleanup(LBK_ERR_DEVICE);
    if ((s = fetch(lat, FLD_SLOTS, 0)) != LBK_OK)
        return cleanup(s);
    if (lat->host[FLD_BAD] != 0.0)
        return cleanup(fail(LBK_ERR_INVALID_ARG,
                            "%.0f field values out of range (need 0<=eps<=1, k>0 or +inf, "
                            "kn0>=0 finite)",
                            lat->host[FLD_BAD]));
    // mean porosity of the pressure columns (for the global permeability)
    lat->eps_b = 0.0;
    if (d->bc_x == LBK_BC_PRESSURE) {
        float *col = nullptr;
        if (hipHostMalloc((void **)&col, 2 * (size_t)d->ny * sizeof(float),
                          hipHostMallocDefault) != hipSuccess)
            return cleanup(fail(LBK_ERR_DEVICE, "pinned host allocation failed"));
        bool ok =
            hip_ok(hipMemcpy2DAsync(col, sizeof(float), med, mrow, sizeof(float), d->ny,
                                    hipMemcpyDeviceToHost, st), "eps column") &&
            hip_ok(hipMemcpy2DAsync(col + d->ny, sizeof(float), med + (d->nx - 1) * sizeof(float),
                                    mrow, sizeof(float), d->ny, hipMemcpyDeviceToHost, st),
                   "eps column") &&
            hip_ok(hipStreamSynchronize(st), "sync");
        double sum = 0.0;
        for (int i = 0; ok && i < 2 * d->ny; ++i)
            sum += col[i];
        (void)hipHostFree(col);
        if (!ok)
            return cleanup(LBK_ERR_DEVICE);
        lat->eps_b = sum / (2.0 * d->ny);
    }
    if (!hip_ok(launch_init_state(d->storage, lat->state(0), L.lay, lat->g, d->init, d->rho0,
                                  d->rho_in, d->rho_out, lat->s(), st), "init kernel") ||
        !hip_ok(hipStreamSynchronize(st), "sync"))
        return cleanup(LBK_ERR_DEVICE);
    *out = lat;
    return LBK_OK;
}

lbk_status lbk_destroy(lbk_lattice *lat)
{
    if (!lat)
        return LBK_OK;
    (void)hipHostFree(lat->host);
    delete lat;
    return LBK_OK;
}

lbk_status lbk_step(lbk_lattice *lat, int64_t n)
{
    if (!lat)
        return fail(LBK_ERR_INVALID_ARG, "lattice is NULL");
    if (n < 0)
        return fail(LBK_ERR_INVALID_ARG, "n must be >= 0");
    const lbk_desc &d = lat->d;
    Range range("lbk_step");
    while (n > 0) {
        // checks fall on multiples of check_every in the lattice's own time,
        // so a run resumed from a saved state checks where the original did
        int64_t chunk = n;
        if (d.check_every > 0)
            chunk = std::min(chunk, d.check_every - lat->t % d.check_every);
        lbk_status s = advance(lat, chunk, lat->stream);
        if (s != LBK_OK)
            return s;
        n -= chunk;
        if (d.check_every > 0 && lat->t % d.check_every == 0 && (s = check_state(lat)) != LBK_OK)
            return s;
    }
    return LBK_OK;
}

lbk_status lbk_time(const lbk_lattice *lat, int64_t *t)
{
    if (!lat || !t)
        return fail(LBK_ERR_INVALID_ARG, "NULL argument");
    *t = lat->t;
    return LBK_OK;
}

lbk_status lbk_steps_per_launch(const lbk_lattice *lat, int32_t *steps)
{
    if (!lat || !steps)
        return fail(LBK_ERR_INVALID_ARG, "NULL argument");
    *steps = three_step_pass(lat) ? 3 : (two_step_pass(lat) ? 2 : 1);
    return LBK_OK;
}

lbk_status lbk_read_macroscopic(lbk_lattice *lat, float *rho, float *ux, float *uy)
{
    if (!lat)
        return fail(LBK_ERR_INVALID_ARG, "lattice is NULL");
    const lbk_desc &d = lat->d;
    HIP_TRY(launch_macro(d.storage, d.bc_x, d.bc_y, lat->state(lat->cur), lat->L.lay,
                         lat->med(), lat->L.mlay, lat->g, lat->ph, lat->s(), lat->inv_s(), rho, ux, uy,
                         nullptr, nullptr, lat->partials(), lat->stream));
    return LBK_OK;
}

lbk_status lbk_read_populations(lbk_lattice *lat, double *f)
{
    if (!lat || !f)
        return fail(LBK_ERR_INVALID_ARG, "NULL argument");
    HIP_TRY(launch_populations(lat->d.storage, lat->state(lat->cur), lat->L.lay, lat->g,
                               lat->inv_s(), f, lat->stream));
    return LBK_OK;
}

} // extern "C"

bool lbk::has_drive(const lbk_desc &d)
{
    return d.bc_x == LBK_BC_PRESSURE ? d.rho_in != d.rho_out : d.gx != 0.0;
}

double lbk::k_app_of(const lbk_lattice *lat, const double *sums)
{
    const lbk_desc &d = lat->d;
    const double n = (double)d.nx * d.ny, nu = (d.tau - 0.5) / 3.0;
    if (!has_drive(d))
        return NAN;
    if (d.bc_x == LBK_BC_PRESSURE)
        return lat->eps_b * nu * (d.nx - 1) * (sums[MAC_FLUX] / n) /
               ((1.0 / 3.0) * (d.rho_in - d.rho_out));
    return nu * (sums[MAC_UX] / n) / d.gx;
}

lbk_status lbk::macro_sums(lbk_lattice *lat, bool residual)
{
    const lbk_desc &d = lat->d;
    char *ws = lat->ws;
    float *uxp = residual ? reinterpret_cast<float *>(ws + lat->L.uxp) : nullptr;
    float *uyp = residual ? reinterpret_cast<float *>(ws + lat->L.uyp) : nullptr;
    HIP_TRY(launch_macro(d.storage, d.bc_x, d.bc_y, lat->state(lat->cur), lat->L.lay,
                         lat->med(), lat->L.mlay, lat->g, lat->ph, lat->s(), lat->inv_s(), nullptr, nullptr,
                         nullptr, uxp, uyp, lat->partials(), lat->stream));
    return fetch(lat, MAC_SLOTS, 0);
}

extern "C" {

lbk_status lbk_apparent_permeability(lbk_lattice *lat, double *k_app)
{
    if (!lat || !k_app)
        return fail(LBK_ERR_INVALID_ARG, "NULL argument");
    if (!has_drive(lat->d))
        return fail(LBK_ERR_INVALID_ARG, "the global permeability needs rho_in != rho_out "
                                         "(pressure drive) or gx != 0");
    lbk_status s = macro_sums(lat, false);
    if (s != LBK_OK)
        return s;
    *k_app = k_app_of(lat, lat->host);
    return LBK_OK;
}

lbk_status lbk_diagnostics(lbk_lattice *lat, double *mass, double *flux_x, double *residual)
{
    if (!lat)
        return fail(LBK_ERR_INVALID_ARG, "lattice is NULL");
    lbk_status s = macro_sums(lat, true);
    if (s != LBK_OK)
        return s;
    const double flux = lat->host[MAC_FLUX];
    // relative change of the velocity field; a field that is zero now and
    // was zero before has not changed (0), one that fell to zero changed
    // by everything it had (+inf)
    const double du2 = lat->host[MAC_DU2], u2 = lat->host[MAC_U2];
    const double res = !lat->have_prev ? INFINITY
                       : u2 > 0.0      ? sqrt(du2 / u2)
                       : du2 > 0.0     ? INFINITY
                                       : 0.0;
    lat->have_prev = true;
    if (flux_x)
        *flux_x = flux;
    if (residual)
        *residual = res;
    if (mass) {
        HIP_TRY(launch_state_sums(lat->d.storage, lat->state(lat->cur), lat->L.lay, lat->g,
                                  lat->inv_s(), lat->partials(), lat->stream));
        if ((s = fetch(lat, ST_SLOTS, 1u << ST_HMAX)) != LBK_OK)
            return s;
        *mass = lat->host[ST_MASS];
    }
    return LBK_OK;
}

// Saved state: a 64-byte header (magic, step count, FP16 scale exponent,
// sizes) followed by the current time level (density and deviations).
static const uint64_t kMagic = 0x6c626b7374617465ull; // "lbkstate"

lbk_status lbk_state_size(const lbk_lattice *lat, size_t *bytes)
{
    if (!lat || !bytes)
        return fail(LBK_ERR_INVALID_ARG, "NULL argument");
    *bytes = 64 + lat->L.level_bytes;
    return LBK_OK;
}

lbk_status lbk_save_state(lbk_lattice *lat, void *dst)
{
    if (!lat || !dst)
        return fail(LBK_ERR_INVALID_ARG, "NULL argument");
    size_t bytes;
    lbk_state_size(lat, &bytes);
    int64_t hdr[8] = {(int64_t)kMagic, lat->t, lat->scale_exp, (int64_t)bytes,
                      lat->d.nx,       lat->d.ny, lat->d.storage, 0};
    HIP_TRY(hipStreamSynchronize(lat->stream));
    HIP_TRY(hipMemcpy(dst, hdr, sizeof hdr, hipMemcpyDefault));
    HIP_TRY(hipMemcpyAsync(static_cast<char *>(dst) + 64, lat->state(lat->cur), bytes - 64,
                           hipMemcpyDefault, lat->stream));
    return LBK_OK;
}

lbk_status lbk_load_state(lbk_lattice *lat, const void *src)
{
    if (!lat || !src)
        return fail(LBK_ERR_INVALID_ARG, "NULL argument");
    size_t bytes;
    lbk_state_size(lat, &bytes);
    int64_t hdr[8];
    HIP_TRY(hipStreamSynchronize(lat->stream));
    HIP_TRY(hipMemcpy(hdr, src, sizeof hdr, hipMemcpyDefault));
    if (hdr[0] != (int64_t)kMagic || hdr[3] != (int64_t)bytes || hdr[4] != lat->d.nx ||
        hdr[5] != lat->d.ny || hdr[6] != lat->d.storage)
        return fail(LBK_ERR_INVALID_ARG, "state does not match this lattice");
    HIP_TRY(hipMemcpyAsync(lat->state(lat->cur), static_cast<const char *>(src) + 64,
                           bytes - 64, hipMemcpyDefault, lat->stream));
    lat->t = hdr[1];
    lat->scale_exp = (int)hdr[2];
    ++lat->version;
    lat->have_prev = false;
    return LBK_OK;
}

lbk_status lbk_correction_factor(int32_t correlation, double slip_b, const double *kn,
                                 double *fc, size_t n)
{
    if ((n && (!kn || !fc)))
        return fail(LBK_ERR_INVALID_ARG, "NULL argument");
    if (correlation < 0 || correlation > 2)
        return fail(LBK_ERR_INVALID_ARG, "correlation must be 0..2 (got %d)", correlation);
    if (!(slip_b <= 0.0) || !isfinite(slip_b))
        return fail(LBK_ERR_INVALID_ARG, "slip_b must be finite and <= 0");
    for (size_t i = 0; i < n; ++i) {
        const double k = kn[i];
        if (!(k >= 0.0) || !isfinite(k))
            return fail(LBK_ERR_INVALID_ARG, "Kn[%zu] = %g is not finite and >= 0", i, k);
        double f = 1.0;
        if (k > 0.0 && correlation == LBK_FC_KLINKENBERG) {
            f = 1.0 + 4.0 * k;
        } else if (k > 0.0 && correlation == LBK_FC_BKC) {
            const double alpha = 1.358 / (1.0 + 0.170 * pow(k, -0.4348));
            f = (1.0 + alpha * k) * (1.0 + 4.0 * k / (1.0 - slip_b * k));
        }
        fc[i] = f;
    }
    return LBK_OK;
}

const char *lbk_last_error(void) { return g_err.c_str(); }

} // extern "C"

// ------------------------------------------------------------ gradients

lbk_status lbk::adj_plan(const lbk_lattice *lat, int64_t n, int64_t c1, int64_t c2,
                         AdjPlan &P)
{
    if (n < 1 || c1 < 1 || c2 < 1 || c2 > c1)
        return fail(LBK_ERR_INVALID_ARG,
                    "need n_steps >= 1 and 1 <= hist_len <= ckpt_every (got %lld, %lld, %lld)",
                    (long long)n, (long long)c1, (long long)c2);
    P = AdjPlan{};
    P.n = n;
    P.c1 = c1;
    P.c2 = c2;
    P.two_level = c2 < c1 && c2 < n;
    P.k1 = (n + c1 - 1) / c1;
    P.k2 = P.two_level ? (c1 + c2 - 1) / c2 : 0;
    P.hlen = P.two_level ? c2 : (c1 < n ? c1 : n);
    const int64_t rows = lat->d.ny;
    P.level_bytes = lat->L.level_bytes;
    P.hist_bytes = (size_t)rows * 3 * lat->L.pitch * 4;
    P.lam_bytes = (size_t)rows * 9 * lat->L.pitch * 4;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes, 256);
        return at;
    };
    P.outer = take(P.level_bytes * (size_t)P.k1);
    P.rec = take(2 * P.level_bytes);
    P.hist = take(P.hist_bytes * (size_t)(P.hlen + 1));
    P.lam = take(2 * P.lam_bytes);
    P.grad = take((size_t)rows * lat->L.pitch * 8);
    P.seg = take((size_t)rows * lat->L.pitch * 4);
    P.grad2 = take((size_t)rows * lat->L.pitch * 8);
    P.seg2 = take((size_t)rows * lat->L.pitch * 4);
    P.inner_seg = P.level_bytes * (size_t)P.k2;
    P.inner = take(P.inner_seg);
    P.keep = P.two_level ? 1 : 0;
    P.total = o;
    return LBK_OK;
}

void lbk::adj_keep(AdjPlan &P, size_t ws_bytes)
{
    if (!P.two_level || ws_bytes < P.total)
        return;
    const size_t extra = (ws_bytes - P.total) / P.inner_seg;
    P.keep = std::min<int64_t>(P.k1, 1 + (int64_t)std::min<size_t>(extra, (size_t)P.k1));
    P.total += (size_t)(P.keep - 1) * P.inner_seg;
}

int64_t lbk::adj_rebuild_steps(const AdjPlan &P)
{
    if (!P.two_level)
        return 0;
    int64_t steps = 0;
    for (int64_t k = 0; k < P.k1 - P.keep; ++k) {
        const int64_t len = std::min(P.c1, P.n - k * P.c1);
        steps += ((len + P.c2 - 1) / P.c2 - 1) * P.c2; // sweep to the last inner start
    }
    return steps;
}

double lbk::objective_weights(const lbk_lattice *lat, int objective, const double *sums,
                              double &a1, double &a2, int &outlet)
{
    const lbk_desc &d = lat->d;
    const double nodes = (double)d.nx * d.ny, nu = (d.tau - 0.5) / 3.0;
    if (objective == LBK_OBJ_OUTLET_FLUX) {
        a1 = 1.0;
        a2 = 0.0;
        outlet = 1;
        return sums[MAC_QOUT];
    }
    outlet = 0;
    if (d.bc_x == LBK_BC_PRESSURE) {
        a1 = lat->eps_b * nu * (d.nx - 1) / ((1.0 / 3.0) * (d.rho_in - d.rho_out) * nodes);
        a2 = 0.0;
        return a1 * sums[MAC_FLUX];
    }
    a1 = 0.0;
    a2 = nu / (d.gx * nodes);
    return a2 * sums[MAC_UX];
}

lbk_status lbk::check_objective(const lbk_lattice *lat, int objective)
{
    const lbk_desc &d = lat->d;
    if (objective != LBK_OBJ_PERMEABILITY && objective != LBK_OBJ_OUTLET_FLUX)
        return fail(LBK_ERR_INVALID_ARG, "unknown objective %d", objective);
    if (objective == LBK_OBJ_PERMEABILITY && !has_drive(d))
        return fail(LBK_ERR_INVALID_ARG, "the global permeability needs rho_in != rho_out "
                                         "(pressure drive) or gx != 0");
    return LBK_OK;
}

extern "C" lbk_status lbk_adjoint_workspace_size(const lbk_lattice *lat, int64_t n_steps,
                                                 int64_t ckpt_every, int64_t hist_len,
                                                 size_t *bytes)
{
    if (!lat || !bytes)
        return fail(LBK_ERR_INVALID_ARG, "NULL argument");
    AdjPlan P;
    lbk_status s = adj_plan(lat, n_steps, ckpt_every, hist_len, P);
    if (s != LBK_OK)
        return s;
    *bytes = P.total;
    return LBK_OK;
}

extern "C" lbk_status lbk_adjoint_plan(const lbk_lattice *lat, int64_t n_steps,
                                       int64_t ckpt_every, size_t budget_bytes,
                                       int64_t *hist_len, size_t *bytes)
{
    if (!lat || !hist_len)
        return fail(LBK_ERR_INVALID_ARG, "NULL argument");
    if (n_steps < 1 || ckpt_every < 1)
        return fail(LBK_ERR_INVALID_ARG, "need n_steps >= 1 and ckpt_every >= 1");
    const int64_t c1 = std::min(ckpt_every, n_steps);
    // fewest sweeps spent rebuilding inner checkpoints; among equals, the
    // longest history (fewest segments)
    int64_t prev = -1, best_h = -1, best_cost = -1;
    size_t best_bytes = 0;
    for (int64_t m = 1; m <= c1; ++m) {
        const int64_t h = (c1 + m - 1) / m;
        if (h == prev)
            continue;
        prev = h;
        AdjPlan P;
        lbk_status s = adj_plan(lat, n_steps, c1, h, P);
        if (s != LBK_OK)
            return s;
        if (P.total > budget_bytes)
            continue;
        adj_keep(P, budget_bytes);
        const int64_t cost = adj_rebuild_steps(P);
        if (best_h < 0 || cost < best_cost) {
            best_h = h;
            best_cost = cost;
            best_bytes = P.total;
        }
        if (cost == 0)
            break;
    }
    if (best_h < 0)
        return fail(LBK_ERR_OOM, "no checkpoint plan for %lld steps every %lld fits in %zu bytes",
                    (long long)n_steps, (long long)c1, budget_bytes);
    *hist_len = best_h;
    if (bytes)
        *bytes = best_bytes;
    return LBK_OK;
}

extern "C" lbk_status lbk_adjoint_forward(lbk_lattice *lat, int objective, int64_t n_steps,
                                          int64_t ckpt_every, int64_t hist_len, void *ws,
                                          size_t ws_bytes, double *J)
{
    if (!lat || !ws || !J)
        return fail(LBK_ERR_INVALID_ARG, "NULL argument");
    Range range("adjoint forward");
    lbk_status s0 = check_objective(lat, objective);
    if (s0 != LBK_OK)
        return s0;
    if ((uintptr_t)ws & 255u)
        return fail(LBK_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
    AdjPlan P;
    lbk_status s = adj_plan(lat, n_steps, ckpt_every, hist_len, P);
    if (s != LBK_OK)
        return s;
    if (ws_bytes < P.total)
        return fail(LBK_ERR_OOM, "adjoint workspace of %zu bytes < %zu needed", ws_bytes,
                    P.total);
    adj_keep(P, ws_bytes);
    lat->adj.valid = false;
    char *w = static_cast<char *>(ws);
    hipStream_t st = lat->stream;
    P.t0 = lat->t;
    for (int64_t k = 0; k < P.k1; ++k) {
        HIP_TRY(hipMemcpyAsync(w + P.outer + (size_t)k * P.level_bytes, lat->state(lat->cur),
                               P.level_bytes, hipMemcpyDeviceToDevice, st));
        const int64_t steps = std::min(P.c1, P.n - k * P.c1);
        // the last `keep` segments are reversed first: keep their inner
        // checkpoints now rather than recomputing them in the backward pass
        const int64_t kept = k - (P.k1 - P.keep);
        const bool keep_inner = P.two_level && kept >= 0;
        const int64_t run = keep_inner ? P.c2 : steps; // steps between kept states
        for (int64_t i = 0; i < steps; i += run) {
            if (keep_inner)
                HIP_TRY(hipMemcpyAsync(w + P.inner + (size_t)kept * P.inner_seg +
                                           (size_t)(i / P.c2) * P.level_bytes,
                                       lat->state(lat->cur), P.level_bytes,
                                       hipMemcpyDeviceToDevice, st));
            if ((s = advance(lat, std::min(run, steps - i), st)) != LBK_OK)
                return s;
        }
    }
    if ((s = macro_sums(lat, false)) != LBK_OK)
        return s;
    P.objective = objective;
    *J = objective_weights(lat, objective, lat->host, P.a1, P.a2, P.outlet);
    P.ws = ws;
    P.valid = true;
    lat->adj = P;
    return LBK_OK;
}

extern "C" lbk_status lbk_adjoint_backward(lbk_lattice *lat, void *ws, size_t ws_bytes,
                                           float *dJ_dlnk, float *dJ_dlnkn0)
{
    if (!lat || !ws || !dJ_dlnk)
        return fail(LBK_ERR_INVALID_ARG, "NULL argument");
    const AdjPlan &P = lat->adj;
    if (!P.valid || P.ws != ws || ws_bytes < P.total)
        return fail(LBK_ERR_INVALID_ARG, "no matching lbk_adjoint_forward for this workspace");
    if (lat->t != P.t0 + P.n)
        return fail(LBK_ERR_INVALID_ARG, "the lattice moved since lbk_adjoint_forward");
    const lbk_desc &d = lat->d;
    hipStream_t st = lat->stream;
    char *w = static_cast<char *>(ws);
    auto level = [&](size_t off, int64_t k) { return w + off + (size_t)k * P.level_bytes; };
    auto histp = [&](int64_t k) {
        return reinterpret_cast<float *>(w + P.hist + (size_t)k * P.hist_bytes);
    };
    float *lam[2] = {reinterpret_cast<float *>(w + P.lam),
                     reinterpret_cast<float *>(w + P.lam + P.lam_bytes)};
    double *grad = reinterpret_cast<double *>(w + P.grad);
    float *seg = reinterpret_cast<float *>(w + P.seg);
    const bool kn = dJ_dlnkn0 != nullptr;
    double *grad2 = reinterpret_cast<double *>(w + P.grad2);
    float *seg2 = kn ? reinterpret_cast<float *>(w + P.seg2) : nullptr;
    char *rec[2] = {level(P.rec, 0), level(P.rec, 1)};
    auto sweep = [&](const char *src, char *dst, float *hist) {
        return launch_sweep(d.storage, d.bc_x, d.bc_y, src, dst, lat->L.lay, lat->med(),
                            lat->L.mlay, lat->g, lat->ph, lat->s(), lat->inv_s(), hist, st);
    };
    // two steps src -> dst in one pass, recording both when hist1 is given;
    // rebuilt inner checkpoints (no history) and recorded segments take
    // lbk_step's passes, the reverse steps pairs
    const bool two = two_step_pass(lat), three = three_step_pass(lat);
    auto sweep2 = [&](const char *src, char *dst, float *hist1, float *hist2) {
        return launch_sweep2(d.storage, d.bc_x, d.bc_y, src, dst, lat->L.lay, lat->med(),
                             lat->L.mlay, lat->g, lat->ph, lat->s(), lat->inv_s(),
                             fwd_band(d), hist1, hist2, st);
    };
    // three steps src -> dst in one pass, recording all three when hist1
    // is given
    auto sweep3 = [&](const char *src, char *dst, float *hist1, float *hist2, float *hist3) {
        return launch_sweep3x(d.storage, d.bc_x, d.bc_y, src, dst, lat->L.lay, lat->med(),
                              lat->L.mlay, lat->g, lat->ph, lat->s(), lat->inv_s(),
                              fwd_band3(d), hist1, hist2, hist3, st);
    };
    const float a1 = (float)P.a1, a2 = (float)P.a2;

    HIP_TRY(hipMemsetAsync(grad, 0, (size_t)d.ny * lat->L.pitch * 8, st));
    HIP_TRY(hipMemsetAsync(seg, 0, (size_t)d.ny * lat->L.pitch * 4, st));
    if (kn) {
        HIP_TRY(hipMemsetAsync(grad2, 0, (size_t)d.ny * lat->L.pitch * 8, st));
        HIP_TRY(hipMemsetAsync(seg2, 0, (size_t)d.ny * lat->L.pitch * 4, st));
    }
    // read-out of J at step n: linearisation point of the pull of S_n
    HIP_TRY(sweep(lat->state(lat->cur), rec[0], histp(0)));
    HIP_TRY(launch_adjoint(d.bc_x, d.bc_y, nullptr, lam[0], histp(0), lat->med(), lat->L.mlay,
                           seg, seg2, lat->g, lat->ph, 1, a1, a2, P.outlet, st));
    int cur = 0;
    for (int64_t k = P.k1 - 1; k >= 0; --k) {
        const int64_t a = k * P.c1, b = std::min(P.n, a + P.c1);
        int64_t nseg = 1;
        // inner checkpoints of this segment: kept by the forward pass, or
        // rebuilt into the first kept segment's slots (free by now, since
        // the kept segments are the last ones and reversed first)
        const int64_t kept = k - (P.k1 - P.keep);
        const size_t inner = P.inner + (size_t)(kept > 0 ? kept : 0) * P.inner_seg;
        if (P.two_level && kept >= 0) {
            nseg = (b - a + P.c2 - 1) / P.c2;
        } else if (P.two_level) {
            // rebuild the inner checkpoints of this outer segment
            Range range("adjoint rebuild");
            const char *src = level(P.outer, k);
            int r = 0;
            nseg = 0;
            for (int64_t t = a; t < b; t += P.c2, ++nseg) {
                HIP_TRY(hipMemcpyAsync(level(inner, nseg), src, P.level_bytes,
                                       hipMemcpyDeviceToDevice, st));
                const int64_t steps = std::min(P.c2, b - t);
                if (t + steps >= b)
                    break; // the last inner segment needs no further state
                for (int64_t i = 0; i < steps;) {
                    const char *from = i == 0 ? level(inner, nseg) : rec[r];
                    if (three && i + 2 < steps) {
                        HIP_TRY(sweep3(from, rec[r ^ 1], nullptr, nullptr, nullptr));
                        i += 3;
                    } else if (two && i + 1 < steps) {
                        HIP_TRY(sweep2(from, rec[r ^ 1], nullptr, nullptr));
                        i += 2;
                    } else {
                        HIP_TRY(sweep(from, rec[r ^ 1], nullptr));
                        ++i;
                    }
                    r ^= 1;
                }
                src = rec[r];
            }
            ++nseg;
        }
        for (int64_t j = nseg - 1; j >= 0; --j) {
            const int64_t a2s = P.two_level ? a + j * P.c2 : a;
            const int64_t b2s = P.two_level ? std::min(b, a2s + P.c2) : b;
            const char *src = P.two_level ? level(inner, j) : level(P.outer, k);
            // recompute the segment, recording each step's linearisation point
            int r = 0;
            {
                Range range("adjoint recompute");
                for (int64_t t = a2s; t < b2s;) {
                    const char *from = t == a2s ? src : rec[r];
                    if (three && t + 2 < b2s) {
                        HIP_TRY(sweep3(from, rec[r ^ 1], histp(t - a2s + 1), histp(t - a2s + 2),
                                       histp(t - a2s + 3)));
                        t += 3;
                    } else if (two && t + 1 < b2s) {
                        HIP_TRY(sweep2(from, rec[r ^ 1], histp(t - a2s + 1), histp(t - a2s + 2)));
                        t += 2;
                    } else {
                        HIP_TRY(sweep(from, rec[r ^ 1], histp(t - a2s + 1)));
                        ++t;
                    }
                    r ^= 1;
                }
            }
            Range range("adjoint reverse");
            for (int64_t t = b2s; t > a2s;) {
                if (two && t - 1 > a2s) {
                    HIP_TRY(launch_adjoint2(d.bc_x, d.bc_y, lam[cur], lam[cur ^ 1],
                                            histp(t - a2s), histp(t - 1 - a2s), lat->med(),
                                            lat->L.mlay, seg, seg2, lat->g, lat->ph,
                                            rev_band(d), st));
                    t -= 2;
                } else {
                    HIP_TRY(launch_adjoint(d.bc_x, d.bc_y, lam[cur], lam[cur ^ 1],
                                           histp(t - a2s), lat->med(), lat->L.mlay, seg, seg2,
                                           lat->g, lat->ph, 0, a1, a2, P.outlet, st));
                    --t;
                }
                cur ^= 1;
            }
            HIP_TRY(launch_grad_fold(seg, grad, lat->g, st));
            if (kn)
                HIP_TRY(launch_grad_fold(seg2, grad2, lat->g, st));
        }
    }
    HIP_TRY(launch_grad_out(grad, dJ_dlnk, lat->g, st));
    if (kn)
        HIP_TRY(launch_grad_out(grad2, dJ_dlnkn0, lat->g, st));
    return LBK_OK;
}
