// lbk_kernels.hip -- HIP kernels (gfx950) of the Klinkenberg lattice
// Boltzmann hot path: the fused pull-stream + Klinkenberg + velocity +
// BGK/Guo collide sweep (one launch per time step, Eq. 12), the macroscopic
// read-out (Eqs. 16-17), deterministic FP64 reductions for the global
// permeability and mass, and field / state set-up.
//
// Layout in HBM (per time level, two levels ping-pong):
//   rho  FP32  [ny][pitch]          node density
//   h    T     [9][ny][pitch]       deviations f*_i - w_i rho (T = FP32/FP16/BF16)
// plus the read-only medium planes eps, drag = eps nu / k, kn0 (FP32).
// pitch is a multiple of 64 elements; x is the fastest index.
//
// Work mapping: one node per thread, 256 threads = 4 wave64s per block, a
// block covers 256 consecutive x of one row.  The 1-D grid is remapped so
// that each of the 8 XCDs (which receive blocks round-robin) sweeps one
// contiguous band of rows: neighbouring rows share the density plane and
// row-edge cache lines in that XCD's L2.
#include "lbk_kernels.h"

namespace lbk {

Launch launch_of(const Geom &g)
{
    Launch l;
    l.blocks_per_row = (g.nx + kBlock - 1) / kBlock;
    l.blocks = l.blocks_per_row * g.ny;
    return l;
}

// Hardware block b lands on XCD b % 8; give XCD j the j-th contiguous chunk
// of logical blocks.  A bijection on [0, nb) for any nb.
__device__ __forceinline__ int xcd_remap(int b, int nb)
{
    const int q = nb >> 3, r = nb & 7;
    const int j = b & 7, idx = b >> 3;
    return j * q + (j < r ? j : r) + idx;
}

// Post-stream deviations of node (x, y) after the boundary override; returns
// the FP32 density the deviations are taken against.
template <typename T, int BCX, int BCY>
__device__ __forceinline__ float post_stream(const State<T> &src, const Geom &g, const Medium &m,
                                             const Physics &ph, float inv_s, int x, int y,
                                             float (&dl)[9])
{
    if (BCX == BC_PRESSURE && (x == 0 || x == g.nx - 1)) {
        // non-equilibrium extrapolation from the neighbouring column:
        // f_i = f_eq_i(rho_b, u_n; eps_b) + f_i(n) - f_eq_i(rho_n, u_n; eps_n)
        const int xn = (x == 0) ? 1 : g.nx - 2;
        float rcn, dn[9], dln[9];
        pull<T, BCX, BCY>(src, g, inv_s, xn, y, rcn, dn);
        const float rhon = split_density(rcn, dn, dln);
        float rn = 0.0f;
#pragma unroll
        for (int i = 0; i < 9; ++i)
            rn += dln[i];
        float jx, jy, ux, uy, Fx, Fy;
        momentum(dln, jx, jy);
        const int cn = y * g.pitch + xn, cb = y * g.pitch + x;
        velocity(ph, rhon, jx, jy, m.eps[cn], m.drag[cn], m.kn0[cn], ux, uy, Fx, Fy);
        const bool in = (x == 0);
        const float rb = in ? ph.rin_hi : ph.rout_hi;
        const float rbl = in ? ph.rin_lo : ph.rout_lo;
        float gb[9], gn[9];
        geq_dev(rb, ux, uy, m.eps[cb], gb);
        geq_dev(rhon, ux, uy, m.eps[cn], gn);
#pragma unroll
        for (int i = 0; i < 9; ++i)
            dl[i] = w_of(i) * (rbl - rn) + gb[i] + (dln[i] - gn[i]);
        return rb;
    }
    float rc, d[9];
    pull<T, BCX, BCY>(src, g, inv_s, x, y, rc, d);
    return split_density(rc, d, dl);
}

template <typename T, int BCX, int BCY>
__global__ __launch_bounds__(kBlock) void sweep_kernel(State<T> src, State<T> dst, Geom g,
                                                        Medium m, Physics ph, float s,
                                                        float inv_s, int bpr)
{
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    const int y = L / bpr;
    const int x = (L - y * bpr) * kBlock + threadIdx.x;
    if (x >= g.nx)
        return;
    float dl[9];
    const float rho = post_stream<T, BCX, BCY>(src, g, m, ph, inv_s, x, y, dl);
    float jx, jy, ux, uy, Fx, Fy;
    momentum(dl, jx, jy);
    const int c = y * g.pitch + x;
    const float eps = m.eps[c];
    velocity(ph, rho, jx, jy, eps, m.drag[c], m.kn0[c], ux, uy, Fx, Fy);
    float hs[9];
    collide(ph, rho, dl, ux, uy, Fx, Fy, eps, hs);
    __builtin_nontemporal_store(rho, dst.rho + c);
#pragma unroll
    for (int i = 0; i < 9; ++i)
        Elem<T>::st(dst.h + i * g.plane, c, hs[i], s);
}

// ----------------------------------------------------------- reductions

struct SumOp {
    static __device__ __forceinline__ double f(double a, double b) { return a + b; }
};
struct MaxOp {
    static __device__ __forceinline__ double f(double a, double b) { return a > b ? a : b; }
};

// Fixed-order block reduction of one value: butterfly inside each wave64,
// then the four wave results in order.  Every thread must call it.
template <typename Op>
__device__ __forceinline__ double block_reduce(double v, double *sh)
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        v = Op::f(v, __shfl_xor(v, off, 64));
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    __syncthreads();
    if (lane == 0)
        sh[wave] = v;
    __syncthreads();
    double r = sh[0];
#pragma unroll
    for (int w = 1; w < kBlock / 64; ++w)
        r = Op::f(r, sh[w]);
    return r;
}

template <typename T, int BCX, int BCY>
__global__ __launch_bounds__(kBlock) void macro_kernel(State<T> src, Geom g, Medium m,
                                                        Physics ph, float inv_s, int bpr,
                                                        float *rho_out, float *ux_out,
                                                        float *uy_out, float *ux_prev,
                                                        float *uy_prev, double *partials)
{
    __shared__ double sh[kBlock / 64];
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    const int y = L / bpr;
    const int x = (L - y * bpr) * kBlock + threadIdx.x;
    double v[MAC_SLOTS] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (x < g.nx) {
        float dl[9];
        const float rho = post_stream<T, BCX, BCY>(src, g, m, ph, inv_s, x, y, dl);
        float jx, jy, ux, uy, Fx, Fy;
        momentum(dl, jx, jy);
        const int c = y * g.pitch + x;
        velocity(ph, rho, jx, jy, m.eps[c], m.drag[c], m.kn0[c], ux, uy, Fx, Fy);
        float r = 0.0f;
#pragma unroll
        for (int i = 0; i < 9; ++i)
            r += dl[i];
        const double rp = (double)rho + (double)r;
        const int o = y * g.nx + x;
        if (rho_out)
            rho_out[o] = (float)rp;
        if (ux_out)
            ux_out[o] = ux;
        if (uy_out)
            uy_out[o] = uy;
        v[MAC_FLUX] = rp * (double)ux;
        v[MAC_UX] = ux;
        v[MAC_U2] = (double)ux * ux + (double)uy * uy;
        v[MAC_RHO] = rp;
        if (ux_prev) {
            const double dx = (double)ux - ux_prev[c], dy = (double)uy - uy_prev[c];
            v[MAC_DU2] = dx * dx + dy * dy;
            ux_prev[c] = ux;
            uy_prev[c] = uy;
        }
    }
#pragma unroll
    for (int k = 0; k < MAC_SLOTS; ++k) {
        const double r = block_reduce<SumOp>(v[k], sh);
        if (threadIdx.x == 0)
            partials[(int64_t)k * gridDim.x + L] = r;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void state_sums_kernel(State<T> src, Geom g, float inv_s,
                                                             int bpr, double *partials)
{
    __shared__ double sh[kBlock / 64];
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    const int y = L / bpr;
    const int x = (L - y * bpr) * kBlock + threadIdx.x;
    double mass = 0.0, hmax = 0.0, bad = 0.0;
    if (x < g.nx) {
        const int c = y * g.pitch + x;
        const float rho = src.rho[c];
        double hs = 0.0;
        bad += isfinite(rho) ? 0.0 : 1.0;
#pragma unroll
        for (int i = 0; i < 9; ++i) {
            const float h = Elem<T>::ld(src.h + i * g.plane, c, inv_s);
            hs += (double)h;
            const double a = fabs((double)h);
            hmax = a > hmax ? a : hmax;
            bad += isfinite(h) ? 0.0 : 1.0;
        }
        mass = (double)rho + hs;
    }
    double r = block_reduce<SumOp>(mass, sh);
    if (threadIdx.x == 0)
        partials[(int64_t)ST_MASS * gridDim.x + L] = r;
    r = block_reduce<MaxOp>(hmax, sh);
    if (threadIdx.x == 0)
        partials[(int64_t)ST_HMAX * gridDim.x + L] = r;
    r = block_reduce<SumOp>(bad, sh);
    if (threadIdx.x == 0)
        partials[(int64_t)ST_BAD * gridDim.x + L] = r;
}

__global__ __launch_bounds__(kBlock) void finish_kernel(const double *partials, int slots,
                                                         int blocks, unsigned max_mask,
                                                         double *out)
{
    __shared__ double sh[kBlock / 64];
    for (int k = 0; k < slots; ++k) {
        const bool is_max = (max_mask >> k) & 1u;
        const double *p = partials + (int64_t)k * blocks;
        double v = 0.0;
        for (int j = threadIdx.x; j < blocks; j += kBlock)
            v = is_max ? (p[j] > v ? p[j] : v) : v + p[j];
        const double r = is_max ? block_reduce<MaxOp>(v, sh) : block_reduce<SumOp>(v, sh);
        if (threadIdx.x == 0)
            out[k] = r;
    }
}

// ---------------------------------------------------------------- set-up

__global__ __launch_bounds__(kBlock) void fields_kernel(Geom g, float *eps, float *drag,
                                                         float *kn0, double nu, int bpr,
                                                         double *partials)
{
    __shared__ double sh[kBlock / 64];
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    const int y = L / bpr;
    const int x = (L - y * bpr) * kBlock + threadIdx.x;
    double bad = 0.0;
    if (x < g.nx) {
        const int c = y * g.pitch + x;
        const float e = eps[c], k = drag[c], kn = kn0[c];
        const bool ok = (e >= 0.0f && e <= 1.0f) && (k > 0.0f) && (kn >= 0.0f) && isfinite(kn);
        bad = ok ? 0.0 : 1.0;
        double d = 0.0;
        if (ok && e > 0.0f && isfinite(k))
            d = (double)e * nu / (double)k;
        drag[c] = (float)d;
    }
    const double r = block_reduce<SumOp>(bad, sh);
    if (threadIdx.x == 0)
        partials[(int64_t)FLD_BAD * gridDim.x + L] = r;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void init_state_kernel(State<T> dst, Geom g, int ramp,
                                                             double rho0, double rho_in,
                                                             double rho_out, float s, int bpr)
{
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    const int y = L / bpr;
    const int x = (L - y * bpr) * kBlock + threadIdx.x;
    if (x >= g.nx)
        return;
    double rho = rho0;
    if (ramp)
        rho = g.nx > 1 ? rho_in + (rho_out - rho_in) * (double)x / (double)(g.nx - 1) : rho_in;
    const float hi = (float)rho;
    const float lo = (float)(rho - (double)hi);
    const int c = y * g.pitch + x;
    dst.rho[c] = hi;
#pragma unroll
    for (int i = 0; i < 9; ++i)
        Elem<T>::st(dst.h + i * g.plane, c, w_of(i) * lo, s);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void populations_kernel(State<T> src, Geom g, float inv_s,
                                                              int bpr, double *out)
{
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    const int y = L / bpr;
    const int x = (L - y * bpr) * kBlock + threadIdx.x;
    if (x >= g.nx)
        return;
    const int c = y * g.pitch + x;
    const double rho = src.rho[c];
    const int64_t n = (int64_t)g.nx * g.ny;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const double w = i == 0 ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0);
        out[i * n + (int64_t)y * g.nx + x] =
            w * rho + (double)Elem<T>::ld(src.h + i * g.plane, c, inv_s);
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void rescale_kernel(State<T> st, Geom g, float f, int bpr)
{
    const int L = xcd_remap(blockIdx.x, gridDim.x);
    const int y = L / bpr;
    const int x = (L - y * bpr) * kBlock + threadIdx.x;
    if (x >= g.nx)
        return;
    const int c = y * g.pitch + x;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        T *p = st.h + i * g.plane;
        Elem<T>::st(p, c, Elem<T>::ld(p, c, 1.0f), f);
    }
}

// ------------------------------------------------------------- launchers

template <typename T> static State<T> typed(const StateV &s)
{
    return State<T>{s.rho, static_cast<T *>(s.h)};
}

template <typename T, int BCX, int BCY>
static hipError_t sweep_t(const StateV &src, const StateV &dst, const Geom &g, const Medium &m,
                          const Physics &ph, float s, float inv_s, hipStream_t st)
{
    const Launch l = launch_of(g);
    hipLaunchKernelGGL((sweep_kernel<T, BCX, BCY>), dim3(l.blocks), dim3(kBlock), 0, st,
                       typed<T>(src), typed<T>(dst), g, m, ph, s, inv_s, l.blocks_per_row);
    return hipGetLastError();
}

template <typename T, int BCX, int BCY>
static hipError_t macro_t(const StateV &src, const Geom &g, const Medium &m, const Physics &ph,
                          float inv_s, float *rho_out, float *ux_out, float *uy_out,
                          float *ux_prev, float *uy_prev, double *partials, hipStream_t st)
{
    const Launch l = launch_of(g);
    hipLaunchKernelGGL((macro_kernel<T, BCX, BCY>), dim3(l.blocks), dim3(kBlock), 0, st,
                       typed<T>(src), g, m, ph, inv_s, l.blocks_per_row, rho_out, ux_out,
                       uy_out, ux_prev, uy_prev, partials);
    return hipGetLastError();
}

// Dispatch a (storage, bc_x, bc_y) triple to a template instance.
#define LBK_DISPATCH_BC(FN, T, ...)                                                          \
    switch (bcx * 2 + bcy) {                                                                 \
    case 0: return FN<T, BC_PERIODIC, BC_PERIODIC>(__VA_ARGS__);                             \
    case 1: return FN<T, BC_PERIODIC, BC_WALL>(__VA_ARGS__);                                 \
    case 2: return FN<T, BC_WALL, BC_PERIODIC>(__VA_ARGS__);                                 \
    case 3: return FN<T, BC_WALL, BC_WALL>(__VA_ARGS__);                                     \
    case 4: return FN<T, BC_PRESSURE, BC_PERIODIC>(__VA_ARGS__);                             \
    case 5: return FN<T, BC_PRESSURE, BC_WALL>(__VA_ARGS__);                                 \
    default: return hipErrorInvalidValue;                                                    \
    }

#define LBK_DISPATCH(FN, ...)                                                                \
    switch (storage) {                                                                       \
    case 0: LBK_DISPATCH_BC(FN, float, __VA_ARGS__)                                          \
    case 1: LBK_DISPATCH_BC(FN, __half, __VA_ARGS__)                                         \
    case 2: LBK_DISPATCH_BC(FN, __hip_bfloat16, __VA_ARGS__)                                 \
    default: return hipErrorInvalidValue;                                                    \
    }

hipError_t launch_sweep(int storage, int bcx, int bcy, const StateV &src, const StateV &dst,
                        const Geom &g, const Medium &m, const Physics &ph, float s, float inv_s,
                        hipStream_t st)
{
    if (bcy < 0 || bcy > 1)
        return hipErrorInvalidValue;
    LBK_DISPATCH(sweep_t, src, dst, g, m, ph, s, inv_s, st)
}

hipError_t launch_macro(int storage, int bcx, int bcy, const StateV &src, const Geom &g,
                        const Medium &m, const Physics &ph, float inv_s, float *rho_out,
                        float *ux_out, float *uy_out, float *ux_prev, float *uy_prev,
                        double *partials, hipStream_t st)
{
    if (bcy < 0 || bcy > 1)
        return hipErrorInvalidValue;
    LBK_DISPATCH(macro_t, src, g, m, ph, inv_s, rho_out, ux_out, uy_out, ux_prev, uy_prev,
                 partials, st)
}

hipError_t launch_state_sums(int storage, const StateV &src, const Geom &g, float inv_s,
                             double *partials, hipStream_t st)
{
    const Launch l = launch_of(g);
    switch (storage) {
    case 0:
        hipLaunchKernelGGL(state_sums_kernel<float>, dim3(l.blocks), dim3(kBlock), 0, st,
                           typed<float>(src), g, inv_s, l.blocks_per_row, partials);
        break;
    case 1:
        hipLaunchKernelGGL(state_sums_kernel<__half>, dim3(l.blocks), dim3(kBlock), 0, st,
                           typed<__half>(src), g, inv_s, l.blocks_per_row, partials);
        break;
    case 2:
        hipLaunchKernelGGL(state_sums_kernel<__hip_bfloat16>, dim3(l.blocks), dim3(kBlock), 0,
                           st, typed<__hip_bfloat16>(src), g, inv_s, l.blocks_per_row,
                           partials);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_finish(const double *partials, int slots, int blocks, unsigned max_mask,
                         double *out, hipStream_t st)
{
    hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(kBlock), 0, st, partials, slots, blocks,
                       max_mask, out);
    return hipGetLastError();
}

hipError_t launch_fields(const Geom &g, float *eps, float *drag, float *kn0, double nu,
                         double *partials, hipStream_t st)
{
    const Launch l = launch_of(g);
    hipLaunchKernelGGL(fields_kernel, dim3(l.blocks), dim3(kBlock), 0, st, g, eps, drag, kn0,
                       nu, l.blocks_per_row, partials);
    return hipGetLastError();
}

hipError_t launch_init_state(int storage, const StateV &dst, const Geom &g, int ramp,
                             double rho0, double rho_in, double rho_out, float s,
                             hipStream_t st)
{
    const Launch l = launch_of(g);
    switch (storage) {
    case 0:
        hipLaunchKernelGGL(init_state_kernel<float>, dim3(l.blocks), dim3(kBlock), 0, st,
                           typed<float>(dst), g, ramp, rho0, rho_in, rho_out, s,
                           l.blocks_per_row);
        break;
    case 1:
        hipLaunchKernelGGL(init_state_kernel<__half>, dim3(l.blocks), dim3(kBlock), 0, st,
                           typed<__half>(dst), g, ramp, rho0, rho_in, rho_out, s,
                           l.blocks_per_row);
        break;
    case 2:
        hipLaunchKernelGGL(init_state_kernel<__hip_bfloat16>, dim3(l.blocks), dim3(kBlock), 0,
                           st, typed<__hip_bfloat16>(dst), g, ramp, rho0, rho_in, rho_out, s,
                           l.blocks_per_row);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_populations(int storage, const StateV &src, const Geom &g, float inv_s,
                              double *out, hipStream_t st)
{
    const Launch l = launch_of(g);
    switch (storage) {
    case 0:
        hipLaunchKernelGGL(populations_kernel<float>, dim3(l.blocks), dim3(kBlock), 0, st,
                           typed<float>(src), g, inv_s, l.blocks_per_row, out);
        break;
    case 1:
        hipLaunchKernelGGL(populations_kernel<__half>, dim3(l.blocks), dim3(kBlock), 0, st,
                           typed<__half>(src), g, inv_s, l.blocks_per_row, out);
        break;
    case 2:
        hipLaunchKernelGGL(populations_kernel<__hip_bfloat16>, dim3(l.blocks), dim3(kBlock), 0,
                           st, typed<__hip_bfloat16>(src), g, inv_s, l.blocks_per_row, out);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_rescale(int storage, const StateV &s_, const Geom &g, int k, hipStream_t st)
{
    const Launch l = launch_of(g);
    const float f = ldexpf(1.0f, k);
    switch (storage) {
    case 0:
        hipLaunchKernelGGL(rescale_kernel<float>, dim3(l.blocks), dim3(kBlock), 0, st,
                           typed<float>(s_), g, f, l.blocks_per_row);
        break;
    case 1:
        hipLaunchKernelGGL(rescale_kernel<__half>, dim3(l.blocks), dim3(kBlock), 0, st,
                           typed<__half>(s_), g, f, l.blocks_per_row);
        break;
    case 2:
        hipLaunchKernelGGL(rescale_kernel<__hip_bfloat16>, dim3(l.blocks), dim3(kBlock), 0, st,
                           typed<__hip_bfloat16>(s_), g, f, l.blocks_per_row);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

} // namespace lbk
