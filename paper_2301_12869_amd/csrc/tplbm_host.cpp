// Host side of the C ABI declared in include/tplbm.h: parameter validation,
// workspace layout, kernel launches, checkpoints, and the FP64
// equation-of-state utilities (critical point, coexistence, spinodals).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/tplbm.h"
#include "eos_host.hpp"
#include "lbm_internal.hpp"

using namespace tplbm;

struct tplbm_ctx {
    tplbm_params p;
    hipStream_t stream = nullptr;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    void *f[2] = {nullptr, nullptr};
    double *T[2] = {nullptr, nullptr};
    double *partials = nullptr;
    StepState *st = nullptr;
    double *M = nullptr, *U = nullptr;  // D3Q19 readout buffers (U also hands u, rho to the energy kernel)
    double *rref = nullptr;   // FP32 deviations: reference density per wall-normal layer
    double *lmass = nullptr;  // per-layer next-level mass of a re-centring
    int nlayers = 0;          // wall-normal layers (ny in 2-D, nz in 3-D)
    int ref_interval = 0;     // steps between re-centrings (0: never)
    int cur = 0;
    int64_t step = 0;
    int nblocks = 0;
    int resident = 0;
    size_t N = 0;
    int Q = 9;
    bool mom = false;  // state carried as moments: D2Q9 (rho, j_x, j_y), D3Q19 (rho, j; a fifth plane for the readout's psi)
    int planes = 9;    // state planes per node between steps (Q, or 3 / 5 with mom)
    Phys phys;
    bool have_state = false;
    std::string err;
};

namespace {

thread_local std::string g_err = "no error";

int fail(tplbm_ctx *c, int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    if (c)
        c->err = buf;
    else
        g_err = buf;
    return code;
}

#define HIP_OK(ctx, expr)                                                                  \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail((ctx), TPLBM_EHIP, "%s: %s", #expr, hipGetErrorString(e_));        \
    } while (0)

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

bool tau_one(const tplbm_params &p)
{
    for (double t : p.tau)
        if (t != 1.0) return false;
    return true;
}

// The moment state applies where the post-collision set is a closed function
// of (rho, u, F): every rate 1 (D2Q9 with all rates 1, D3Q19 always); FP64 so
// that it carries exactly what the population state would.
bool moments_apply(const tplbm_params &p)
{
    return (p.lattice == TPLBM_D2Q9 || p.lattice == TPLBM_D3Q19) && p.precision == TPLBM_FP64 && tau_one(p);
}

// AUTO takes the faster state, the moments wherever they apply (D2Q9's row
// march and D3Q19's z march move 64 and 80 B per node-step against 160 and
// 320 for the FP64 populations); MOMENTS asks for them, POPULATIONS not.
bool uses_moments(const tplbm_params &p)
{
    return (p.state == TPLBM_STATE_MOMENTS || p.state == TPLBM_STATE_AUTO) && moments_apply(p);
}

int validate(const tplbm_params *p)
{
    if (!p) return fail(nullptr, TPLBM_EINVAL, "params is NULL");
    if (p->lattice != TPLBM_D2Q9 && p->lattice != TPLBM_D3Q19)
        return fail(nullptr, TPLBM_EINVAL, "lattice must be TPLBM_D2Q9 or TPLBM_D3Q19 (columns use tplbm_batch_*)");
    if (p->lattice == TPLBM_D3Q19) {
        if (p->nx < 1 || p->ny < 1 || p->nz < 3) return fail(nullptr, TPLBM_ESHAPE, "need nx, ny >= 1 and nz >= 3");
        // population indices are 32-bit: 19 N < 2^32
        if ((int64_t)p->nx * p->ny * p->nz * 19 >= (int64_t)1 << 32)
            return fail(nullptr, TPLBM_ESHAPE, "lattice too large (at most 2^32 / 19 nodes)");
        if (!tau_one(*p)) return fail(nullptr, TPLBM_EUNSUPPORTED, "D3Q19 supports only every tau = 1");
    } else {
        if (p->nx < 1 || p->ny < 3) return fail(nullptr, TPLBM_ESHAPE, "need nx >= 1 and ny >= 3");
        if ((int64_t)p->nx * p->ny > (int64_t)1 << 31) return fail(nullptr, TPLBM_ESHAPE, "lattice too large");
    }
    if (p->precision != TPLBM_FP64 && p->precision != TPLBM_FP32_DEV)
        return fail(nullptr, TPLBM_EINVAL, "precision must be TPLBM_FP64 or TPLBM_FP32_DEV");
    if (p->eos != TPLBM_EOS_CARNAHAN_STARLING && p->eos != TPLBM_EOS_IDEAL_LATTICE)
        return fail(nullptr, TPLBM_EINVAL, "unknown eos");
    if (p->gravity_form < 1 || p->gravity_form > 3)
        return fail(nullptr, TPLBM_EINVAL, "gravity_form must be 1, 2 or 3");
    if (!std::isfinite(p->rho_v)) return fail(nullptr, TPLBM_EINVAL, "rho_v must be finite");
    for (int k = 0; k < 6; ++k)
        if (!(p->tau[k] > 0.5)) return fail(nullptr, TPLBM_EINVAL, "tau[%d] must exceed 1/2", k);
    if (p->eos == TPLBM_EOS_CARNAHAN_STARLING) {
        if (!(p->G < 0)) return fail(nullptr, TPLBM_EINVAL, "G must be negative for the Carnahan-Starling pseudopotential");
        if (!(p->a > 0 && p->b > 0 && p->R > 0)) return fail(nullptr, TPLBM_EINVAL, "a, b, R must be positive");
    } else if (p->G == 0) {
        return fail(nullptr, TPLBM_EINVAL, "G must be nonzero");
    }
    if (!(p->cv > 0) || !(p->kappa >= 0)) return fail(nullptr, TPLBM_EINVAL, "need c_v > 0, kappa >= 0");
    if (!std::isfinite(p->g) || !std::isfinite(p->sigma)) return fail(nullptr, TPLBM_EINVAL, "g and sigma must be finite");
    if (p->state != TPLBM_STATE_AUTO && p->state != TPLBM_STATE_POPULATIONS && p->state != TPLBM_STATE_MOMENTS)
        return fail(nullptr, TPLBM_EINVAL,
                    "state must be TPLBM_STATE_AUTO, TPLBM_STATE_POPULATIONS or TPLBM_STATE_MOMENTS");
    if (p->state == TPLBM_STATE_MOMENTS && !moments_apply(*p))
        return fail(nullptr, TPLBM_EINVAL,
                    "the moment state needs a D2Q9 or D3Q19 lattice in FP64 with every relaxation time 1");
    if (p->precision == TPLBM_FP32_DEV && p->ref_interval < 0 && !std::isfinite(p->rho_ref))
        return fail(nullptr, TPLBM_EINVAL, "rho_ref must be finite");
    return TPLBM_OK;
}

Phys make_phys(const tplbm_params &p)
{
    Phys c;
    std::memset(&c, 0, sizeof c);
    c.a = p.a;
    c.b_quarter = p.b / 4.0;
    c.R = p.R;
    c.two_over_G = 2.0 / p.G;
    c.G = p.G;
    c.G2 = p.G * p.G;
    c.sigma = p.sigma;
    c.kappa_over_cv = p.kappa / p.cv;
    c.R_over_cv = p.R / p.cv;
    c.g = p.g;
    c.rho_v = p.rho_v;
    const double t[9] = {p.tau[0], p.tau[1], p.tau[2], p.tau[3], p.tau[4],
                         p.tau[3], p.tau[4], p.tau[5], p.tau[5]};
    for (int k = 0; k < 9; ++k) c.lam[k] = 1.0 / t[k];
    c.sig_e = p.sigma / p.tau[1];
    c.sig_s = p.sigma / p.tau[2];
    c.eos = p.eos;
    c.form = p.gravity_form;
    return c;
}

struct Layout {
    size_t f_bytes, T_bytes, part_bytes, st_bytes, pass_bytes, ref_bytes, total;
    int nblocks;
};

int layers_of(const tplbm_params &p) { return p.lattice == TPLBM_D3Q19 ? p.nz : p.ny; }

size_t nodes_of(const tplbm_params &p)
{
    return (size_t)p.nx * p.ny * (p.lattice == TPLBM_D3Q19 ? (size_t)p.nz : 1);
}
int q_of(const tplbm_params &p) { return p.lattice == TPLBM_D3Q19 ? 19 : 9; }

Layout layout_of(const tplbm_params &p)
{
    Layout L;
    const size_t N = nodes_of(p);
    const size_t elem = p.precision == TPLBM_FP32_DEV ? 4 : 8;
    L.f_bytes = align256(q_of(p) * N * elem);
    L.T_bytes = align256(N * 8);
    if (p.lattice == TPLBM_D3Q19) {
        // readout buffers: M (rho, j, psi), U (u, F, sigma |F_int|^2 / psi^2;
        // a step hands u and rho from the LBM kernel to the energy kernel in
        // its first 4 planes); the moment state is M itself (5 planes: rho,
        // j and the readout's psi) and needs no separate M
        const bool mom = uses_moments(p);
        if (mom) L.f_bytes = align256(5 * N * 8);
        L.pass_bytes = (mom ? 0 : align256(5 * N * 8)) + align256(7 * N * 8);
        L.nblocks = d3q19_num_blocks(p.nx, p.ny, p.nz, 1 << 20);
    } else {
        // the moment state holds 3 planes; the readout scratch reuses the
        // idle state buffer and needs 4N doubles
        if (uses_moments(p)) L.f_bytes = align256(3 * N * 8);
        if (L.f_bytes < align256(4 * N * 8)) L.f_bytes = align256(4 * N * 8);
        L.pass_bytes = 0;
        // partials for the largest grid the persistent launch can use
        L.nblocks = d2q9_num_blocks(p.nx, p.ny, 1 << 20, uses_moments(p));
    }
    L.part_bytes = align256((size_t)L.nblocks * 5 * 8);
    L.st_bytes = align256(sizeof(StepState));
    // FP32 deviations: layer references and the re-centring's layer shares
    L.ref_bytes = p.precision == TPLBM_FP32_DEV ? 2 * align256((size_t)layers_of(p) * 8) : 0;
    L.total = 2 * L.f_bytes + 2 * L.T_bytes + L.part_bytes + L.st_bytes + L.pass_bytes + L.ref_bytes;
    return L;
}

// Compute units of the current device (the persistent grid is sized from it).
int resident_blocks()
{
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        return 256;
    return cus;
}

LatticeLaunch launch_of(tplbm_ctx *c)
{
    LatticeLaunch L;
    L.fin = c->f[c->cur];
    L.fout = c->f[1 - c->cur];
    L.Tin = c->T[c->cur];
    L.Tout = c->T[1 - c->cur];
    L.phys = c->phys;
    L.nx = c->p.nx;
    L.ny = c->p.ny;
    L.nz = c->p.lattice == TPLBM_D3Q19 ? c->p.nz : 1;
    L.fp32 = c->p.precision == TPLBM_FP32_DEV;
    L.tau1 = tau_one(c->p);
    L.walls = c->p.walls != 0;
    L.moments = c->mom;
    L.resident = c->resident;
    L.partials = c->partials;
    L.st = c->st;
    L.step = c->step;
    L.stream = c->stream;
    L.rref = c->rref;
    return L;
}

// The per-layer reference kernels' view of the velocity set.
LayerSet layer_set(const tplbm_params &p)
{
    LayerSet q;
    std::memset(&q, 0, sizeof q);
    if (p.lattice == TPLBM_D3Q19) {
        q.Q = 19;
        for (int i = 0; i < 19; ++i) {
            q.w[i] = i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
            q.cn[i] = kD3Q19z[i];
        }
    } else {
        const double w[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
        const int cy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
        q.Q = 9;
        for (int i = 0; i < 9; ++i) {
            q.w[i] = w[i];
            q.cn[i] = cy[i];
        }
    }
    return q;
}

// D2Q9 velocity set in the paper's order (Eq. VelocitySet) and weights.
const int kCx[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
const int kCy[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
const double kW[9] = {4.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 9, 1.0 / 36, 1.0 / 36, 1.0 / 36, 1.0 / 36};

}  // namespace

extern "C" {

int tplbm_workspace_bytes(const tplbm_params *p, size_t *bytes)
{
    int rc = validate(p);
    if (rc) return rc;
    if (!bytes) return fail(nullptr, TPLBM_EINVAL, "bytes is NULL");
    *bytes = layout_of(*p).total;
    return TPLBM_OK;
}

int tplbm_create(const tplbm_params *p, void *dev_workspace, size_t bytes, void *hip_stream,
                 tplbm_ctx **out)
{
    int rc = validate(p);
    if (rc) return rc;
    if (!out) return fail(nullptr, TPLBM_EINVAL, "out is NULL");
    if (!dev_workspace) return fail(nullptr, TPLBM_EINVAL, "workspace is NULL");
    if (((uintptr_t)dev_workspace & 255) != 0) return fail(nullptr, TPLBM_EINVAL, "workspace must be 256-byte aligned");
    const Layout L = layout_of(*p);
    if (bytes < L.total) return fail(nullptr, TPLBM_ESHAPE, "workspace has %zu bytes, need %zu", bytes, L.total);
    tplbm_ctx *c = new tplbm_ctx();
    c->p = *p;
    c->stream = (hipStream_t)hip_stream;
    c->ws = (char *)dev_workspace;
    c->ws_bytes = bytes;
    c->resident = resident_blocks();
    c->N = nodes_of(*p);
    c->Q = q_of(*p);
    c->mom = uses_moments(*p);
    c->planes = c->mom ? (p->lattice == TPLBM_D3Q19 ? 5 : 3) : c->Q;
    c->nblocks = L.nblocks;
    char *q = c->ws;
    c->f[0] = q; q += L.f_bytes;
    c->f[1] = q; q += L.f_bytes;
    c->T[0] = (double *)q; q += L.T_bytes;
    c->T[1] = (double *)q; q += L.T_bytes;
    c->partials = (double *)q; q += L.part_bytes;
    c->st = (StepState *)q; q += L.st_bytes;
    if (p->lattice == TPLBM_D3Q19) {
        if (!c->mom) { c->M = (double *)q; q += align256(5 * c->N * 8); }
        c->U = (double *)q; q += align256(7 * c->N * 8);
    }
    c->nlayers = layers_of(*p);
    if (p->precision == TPLBM_FP32_DEV) {
        c->rref = (double *)q; q += align256((size_t)c->nlayers * 8);
        c->lmass = (double *)q;
        c->ref_interval = p->ref_interval > 0 ? p->ref_interval
                          : (p->ref_interval == 0 ? TPLBM_REF_INTERVAL_DEFAULT : 0);
    }
    c->phys = make_phys(*p);
    StepState s;
    std::memset(&s, 0, sizeof s);
    s.first_bad = -1;
    hipError_t e = hipMemcpyAsync(c->st, &s, sizeof s, hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) {
        delete c;
        return fail(nullptr, TPLBM_EHIP, "initialising the step state: %s", hipGetErrorString(e));
    }
    *out = c;
    return TPLBM_OK;
}

int tplbm_set_state(tplbm_ctx *c, const double *rho0, const double *T0)
{
    if (!c) return fail(nullptr, TPLBM_EINVAL, "ctx is NULL");
    if (!rho0 || !T0) return fail(c, TPLBM_EINVAL, "rho0 and T0 must be non-NULL");
    const bool d3 = c->p.lattice == TPLBM_D3Q19;
    const int nx = c->p.nx, ny = c->p.ny, nz = d3 ? c->p.nz : 1, Q = c->Q;
    const size_t N = c->N;
    const bool walls = c->p.walls != 0, fp32 = c->p.precision == TPLBM_FP32_DEV;
    // FP32 deviations: one reference density per wall-normal layer, the
    // layer's mean initial density (summed in index order), or the single
    // rho_ref when the references are not re-centred
    const int nl = c->nlayers;
    const size_t lnodes = N / (size_t)nl;
    std::vector<double> rref;
    if (fp32) {
        rref.assign(nl, c->p.rho_ref);
        if (c->p.ref_interval >= 0)
            for (int l = 0; l < nl; ++l) {
                double s = 0.0;
                for (size_t k = 0; k < lnodes; ++k) s += rho0[(size_t)l * lnodes + k];
                rref[l] = s / (double)lnodes;
            }
    }
    double w[19];
    int cx[19], cy[19], cz[19];
    for (int i = 0; i < Q; ++i) {
        if (d3) {
            cx[i] = kD3Q19x[i]; cy[i] = kD3Q19y[i]; cz[i] = kD3Q19z[i];
            w[i] = i == 0 ? 1.0 / 3.0 : (i < 7 ? 1.0 / 18.0 : 1.0 / 36.0);
        } else {
            cx[i] = kCx[i]; cy[i] = kCy[i]; cz[i] = 0;
            w[i] = kW[i];
        }
    }
    // The buffer holds post-collision populations that the first step pulls
    // from: f*_i(x) = w_i rho0(x + c_i) makes the pulled level-0 state the
    // rest state f_i = w_i rho0(x).  Sources beyond a wall are never pulled.
    // The wall-normal axis is y in 2-D and z in 3-D.
    std::vector<double> fd;
    std::vector<float> ff;
    if (c->mom && d3) {
        // As below for D3Q19: rho and j of the pulled rest set, summed in the
        // kernels' order (velocity components of zero add nothing); the psi
        // plane is filled on the device once T^0 is there.
        fd.assign(5 * N, 0.0);
        for (size_t n = 0; n < N; ++n) {
#pragma clang fp contract(off)
            double r = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
            for (int i = 0; i < 19; ++i) {
                const double f = w[i] * rho0[n];
                r += f;
                if (cx[i]) jx += cx[i] * f;
                if (cy[i]) jy += cy[i] * f;
                if (cz[i]) jz += cz[i] * f;
            }
            fd[n] = r;
            fd[N + n] = jx;
            fd[2 * N + n] = jy;
            fd[3 * N + n] = jz;
        }
    } else if (c->mom) {
        // The pulled level-0 set is f_i = w_i rho0(x) at every node (the
        // wall reconstruction returns the same values): store its density
        // and momentum, summed as the kernels sum a pulled set.
        fd.resize(3 * N);
        for (size_t n = 0; n < N; ++n) {
            // the kernels add loaded values: no product may fuse into a sum here
#pragma clang fp contract(off)
            double f[9];
            for (int i = 0; i < 9; ++i) f[i] = w[i] * rho0[n];
            fd[n] = ((f[0] + f[1]) + (f[2] + f[3])) + ((f[4] + f[5]) + (f[6] + f[7])) + f[8];
            fd[N + n] = (f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7]);
            fd[2 * N + n] = (f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8]);
        }
    } else if (fp32) {
        ff.resize((size_t)Q * N);
    } else {
        fd.resize((size_t)Q * N);
    }
    for (int z = 0; z < nz && !c->mom; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const size_t n = ((size_t)z * ny + y) * nx + x;
                for (int i = 0; i < Q; ++i) {
                    int xs = ((x + cx[i]) % nx + nx) % nx;
                    int ys = y + cy[i], zs = z + cz[i];
                    if (d3) {
                        ys = ((ys % ny) + ny) % ny;
                        if (walls) { if (zs < 0 || zs >= nz) zs = z; } else zs = ((zs % nz) + nz) % nz;
                    } else {
                        if (walls) { if (ys < 0 || ys >= ny) ys = y; } else ys = ((ys % ny) + ny) % ny;
                    }
                    const double v = w[i] * rho0[((size_t)zs * ny + ys) * nx + xs];
                    const size_t k = (size_t)i * N + n;
                    if (fp32) ff[k] = (float)(v - w[i] * rref[d3 ? z : y]); else fd[k] = v;
                }
            }
    // <rho> of level 0 from the values the first step will see, index order:
    // with FP32 deviations, population i of node n was stored in the layer
    // of n - c_i (a node's own layer where that lies beyond a wall)
    double tot = 0.0;
    for (size_t n = 0; n < N; ++n) {
        if (fp32) {
            const int l = (int)(n / lnodes);
            double r = 0.0;
            for (int i = 0; i < Q; ++i) {
                int ls = l - (d3 ? cz[i] : cy[i]);
                if (ls < 0 || ls >= nl) ls = walls ? l : (ls + nl) % nl;
                r += w[i] * rref[ls] + (double)(float)(w[i] * rho0[n] - w[i] * rref[ls]);
            }
            tot += r;
        } else {
            tot += rho0[n];
        }
    }
    c->cur = 0;
    c->step = 0;
    if (fp32)
        HIP_OK(c, hipMemcpyAsync(c->f[0], ff.data(), (size_t)Q * N * 4, hipMemcpyHostToDevice, c->stream));
    else
        HIP_OK(c, hipMemcpyAsync(c->f[0], fd.data(), fd.size() * 8, hipMemcpyHostToDevice, c->stream));
    HIP_OK(c, hipMemcpyAsync(c->T[0], T0, N * 8, hipMemcpyHostToDevice, c->stream));
    if (fp32) HIP_OK(c, hipMemcpyAsync(c->rref, rref.data(), (size_t)nl * 8, hipMemcpyHostToDevice, c->stream));
    if (c->mom && d3) {
        LatticeLaunch L = launch_of(c);
        HIP_OK(c, d3q19_launch_psi_init(L, (double *)c->f[0]));
    }
    StepState s;
    std::memset(&s, 0, sizeof s);
    s.mean[0] = tot / (double)N;
    s.mass = tot;
    s.first_bad = -1;
    HIP_OK(c, hipMemcpyAsync(c->st, &s, sizeof s, hipMemcpyHostToDevice, c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    c->have_state = true;
    return TPLBM_OK;
}

int tplbm_step_async(tplbm_ctx *c, int64_t nsteps)
{
    if (!c) return fail(nullptr, TPLBM_EINVAL, "ctx is NULL");
    if (nsteps < 0) return fail(c, TPLBM_EINVAL, "nsteps must be >= 0");
    if (!c->have_state) return fail(c, TPLBM_EINVAL, "call tplbm_set_state or tplbm_load_state first");
    const LayerSet lset = layer_set(c->p);
    for (int64_t s = 0; s < nsteps; ++s) {
        if (c->ref_interval > 0 && c->step > 0 && c->step % c->ref_interval == 0)
            HIP_OK(c, recentre_layers_launch((float *)c->f[c->cur], c->rref, c->lmass, c->N, (int)(c->N / c->nlayers),
                                             c->nlayers, lset, c->p.walls != 0, c->st, (int)(c->step & 1),
                                             c->stream));
        LatticeLaunch L = launch_of(c);
        if (c->p.lattice == TPLBM_D3Q19)
            HIP_OK(c, d3q19_launch_step(L, c->U));
        else
            HIP_OK(c, d2q9_launch_step(L));
        c->cur = 1 - c->cur;
        c->step += 1;
    }
    return TPLBM_OK;
}

int tplbm_step(tplbm_ctx *c, int64_t nsteps)
{
    int rc = tplbm_step_async(c, nsteps);
    if (rc) return rc;
    StepState s;
    HIP_OK(c, hipMemcpyAsync(&s, c->st, sizeof s, hipMemcpyDeviceToHost, c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    if (s.flags)
        return fail(c, TPLBM_EUNPHYSICAL, "unphysical state (flags 0x%x) first seen at level %lld",
                    s.flags, (long long)s.first_bad);
    return TPLBM_OK;
}

int tplbm_read_device(tplbm_ctx *c, int field, double *dev_out)
{
    if (!c) return fail(nullptr, TPLBM_EINVAL, "ctx is NULL");
    if (!dev_out) return fail(c, TPLBM_EINVAL, "output is NULL");
    if (field < TPLBM_RHO || field > TPLBM_P_NN) return fail(c, TPLBM_EINVAL, "unknown field %d", field);
    if (!c->have_state) return fail(c, TPLBM_EINVAL, "no state");
    LatticeLaunch L = launch_of(c);
    if (c->p.lattice == TPLBM_D3Q19)
        HIP_OK(c, d3q19_launch_readout(L, field, c->M, c->U, dev_out));
    else
        HIP_OK(c, d2q9_launch_readout(L, field, (double *)c->f[1 - c->cur], dev_out));
    return TPLBM_OK;
}

int tplbm_read(tplbm_ctx *c, int field, double *host_out)
{
    if (!c) return fail(nullptr, TPLBM_EINVAL, "ctx is NULL");
    if (!host_out) return fail(c, TPLBM_EINVAL, "output is NULL");
    // the readout writes its result into the tail of the idle population
    // buffer (past the 4N-double scratch it uses), then it is copied out
    if (field < TPLBM_RHO || field > TPLBM_P_NN) return fail(c, TPLBM_EINVAL, "unknown field %d", field);
    if (!c->have_state) return fail(c, TPLBM_EINVAL, "no state");
    double *scratch = (double *)c->f[1 - c->cur];
    double *dst = c->T[1 - c->cur];  // idle temperature buffer, N doubles
    LatticeLaunch L = launch_of(c);
    if (c->p.lattice == TPLBM_D3Q19)
        HIP_OK(c, d3q19_launch_readout(L, field, c->M, c->U, dst));
    else
        HIP_OK(c, d2q9_launch_readout(L, field, scratch, dst));
    HIP_OK(c, hipMemcpyAsync(host_out, dst, c->N * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    return TPLBM_OK;
}

int tplbm_diagnostics(tplbm_ctx *c, tplbm_diag *out)
{
    if (!c || !out) return fail(c, TPLBM_EINVAL, "NULL argument");
    StepState s;
    HIP_OK(c, hipMemcpyAsync(&s, c->st, sizeof s, hipMemcpyDeviceToHost, c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    out->step = c->step;
    out->first_bad_step = s.first_bad;
    out->mass = s.mass;
    out->mean_rho = s.mean[c->step & 1];
    out->max_u = s.max_u;
    out->min_rho = s.min_rho;
    out->flags = s.flags;
    out->pad = 0;
    return TPLBM_OK;
}

int tplbm_state_bytes(const tplbm_ctx *c, size_t *bytes)
{
    if (!c || !bytes) return fail(nullptr, TPLBM_EINVAL, "NULL argument");
    const size_t elem = c->p.precision == TPLBM_FP32_DEV ? 4 : 8;
    *bytes = 64 + (size_t)c->planes * c->N * elem + c->N * 8 + sizeof(StepState) + (c->rref ? (size_t)c->nlayers * 8 : 0);
    return TPLBM_OK;
}

namespace {
struct BlobHeader {
    char magic[8];
    int64_t step;
    int64_t N;
    int32_t Q, elem;  // state planes per node and bytes per value
    int32_t nx, ny;
    int32_t lattice, nz, precision, walls;
    char pad[8];
};
static_assert(sizeof(BlobHeader) == 64, "blob header");
}  // namespace

int tplbm_save_state(tplbm_ctx *c, void *host_blob)
{
    if (!c || !host_blob) return fail(c, TPLBM_EINVAL, "NULL argument");
    if (!c->have_state) return fail(c, TPLBM_EINVAL, "no state");
    const size_t elem = c->p.precision == TPLBM_FP32_DEV ? 4 : 8;
    BlobHeader h;
    std::memset(&h, 0, sizeof h);
    std::memcpy(h.magic, "TPLBMST2", 8);
    h.step = c->step;
    h.N = (int64_t)c->N;
    h.Q = c->planes;
    h.elem = (int32_t)elem;
    h.nx = c->p.nx;
    h.ny = c->p.ny;
    h.lattice = c->p.lattice;
    h.nz = c->p.lattice == TPLBM_D3Q19 ? c->p.nz : 1;
    h.precision = c->p.precision;
    h.walls = c->p.walls != 0;
    char *b = (char *)host_blob;
    std::memcpy(b, &h, sizeof h);
    const size_t fb = (size_t)c->planes * c->N * elem;
    HIP_OK(c, hipMemcpyAsync(b + 64, c->f[c->cur], fb, hipMemcpyDeviceToHost, c->stream));
    HIP_OK(c, hipMemcpyAsync(b + 64 + fb, c->T[c->cur], c->N * 8, hipMemcpyDeviceToHost, c->stream));
    HIP_OK(c, hipMemcpyAsync(b + 64 + fb + c->N * 8, c->st, sizeof(StepState),
                             hipMemcpyDeviceToHost, c->stream));
    if (c->rref)
        HIP_OK(c, hipMemcpyAsync(b + 64 + fb + c->N * 8 + sizeof(StepState), c->rref, (size_t)c->nlayers * 8,
                                 hipMemcpyDeviceToHost, c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    return TPLBM_OK;
}

int tplbm_load_state(tplbm_ctx *c, const void *host_blob, size_t bytes)
{
    if (!c || !host_blob) return fail(c, TPLBM_EINVAL, "NULL argument");
    const size_t elem = c->p.precision == TPLBM_FP32_DEV ? 4 : 8;
    size_t want = 0;
    tplbm_state_bytes(c, &want);
    if (bytes != want)
        return fail(c, TPLBM_ESHAPE, "checkpoint has %zu bytes, this lattice's has %zu", bytes, want);
    BlobHeader h;
    std::memcpy(&h, host_blob, sizeof h);
    if (std::memcmp(h.magic, "TPLBMST2", 8) != 0)
        return fail(c, TPLBM_EINVAL, "not a checkpoint of this library (bad magic)");
    if (h.N != (int64_t)c->N || h.elem != (int32_t)elem || h.nx != c->p.nx || h.ny != c->p.ny ||
        h.Q != c->planes || h.lattice != c->p.lattice || h.nz != (c->p.lattice == TPLBM_D3Q19 ? c->p.nz : 1) ||
        h.precision != c->p.precision || h.walls != (c->p.walls != 0))
        return fail(c, TPLBM_ESHAPE, "checkpoint does not match this lattice");
    const char *b = (const char *)host_blob;
    c->cur = 0;
    c->step = h.step;
    const size_t fb = (size_t)c->planes * c->N * elem;
    HIP_OK(c, hipMemcpyAsync(c->f[0], b + 64, fb, hipMemcpyHostToDevice, c->stream));
    HIP_OK(c, hipMemcpyAsync(c->T[0], b + 64 + fb, c->N * 8, hipMemcpyHostToDevice, c->stream));
    StepState s;
    std::memcpy(&s, b + 64 + fb + c->N * 8, sizeof s);
    s.counter = 0;
    HIP_OK(c, hipMemcpyAsync(c->st, &s, sizeof s, hipMemcpyHostToDevice, c->stream));
    if (c->rref)
        HIP_OK(c, hipMemcpyAsync(c->rref, b + 64 + fb + c->N * 8 + sizeof(StepState), (size_t)c->nlayers * 8,
                                 hipMemcpyHostToDevice, c->stream));
    HIP_OK(c, hipStreamSynchronize(c->stream));
    c->have_state = true;
    return TPLBM_OK;
}

void tplbm_destroy(tplbm_ctx *c) { delete c; }

const char *tplbm_last_error(const tplbm_ctx *c) { return c ? c->err.c_str() : g_err.c_str(); }

}  // extern "C"

// FP64 equation-of-state utilities (eos_host.hpp).
using namespace tplbm::eos;

extern "C" int tplbm_eos_critical(double a, double b, double R, double *out3)
{
    if (!out3 || !(a > 0 && b > 0 && R > 0)) return fail(nullptr, TPLBM_EINVAL, "bad EOS constants");
    if (cs_critical(CS{a, b, R}, out3[0], out3[1], out3[2]))
        return fail(nullptr, TPLBM_ENOTCONVERGED, "critical point not bracketed");
    return TPLBM_OK;
}

extern "C" int tplbm_eos_spinodal(double a, double b, double R, double T, double *out2)
{
    if (!out2 || !(a > 0 && b > 0 && R > 0 && T > 0)) return fail(nullptr, TPLBM_EINVAL, "bad arguments");
    CS m{a, b, R};
    double sv, sl;
    int rc = cs_spinodal(m, T, sv, sl);
    if (rc) return fail(nullptr, rc, "no spinodal at T = %g (at or above T_c?)", T);
    out2[0] = sv;
    out2[1] = sl;
    return TPLBM_OK;
}

extern "C" int tplbm_eos_coexistence(double a, double b, double R, double T, double *out3)
{
    if (!out3 || !(a > 0 && b > 0 && R > 0 && T > 0)) return fail(nullptr, TPLBM_EINVAL, "bad arguments");
    double rv, rl, ps;
    int rc = cs_coexistence(CS{a, b, R}, T, rv, rl, ps);
    if (rc == TPLBM_EINVAL) return fail(nullptr, rc, "no coexistence at T = %g (at or above T_c?)", T);
    if (rc) return fail(nullptr, rc, "branch root failed");
    out3[0] = rv;
    out3[1] = rl;
    out3[2] = ps;
    return TPLBM_OK;
}
