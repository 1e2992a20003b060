// C-ABI of the learned two-level preconditioner: handle lifetime, binding to an operator
// (coarse p=1 operator and its probed stencil, log-kappa tiles, multiplicities),
// application z = M(r), loss/gradient, Adam training step and parameter files.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <memory>
#include <random>
#include <vector>

#include "capi_util.h"
#include "internal.h"
#include "k_nn.h"
#include "k_vec.h"

using namespace hexpa;

struct pa_lp {
    pa_lp_opts o{};
    pa_op *op = nullptr;        // bound operator (not owned)
    pa_op *coarse = nullptr;    // p = 1 operator on the same mesh (owned)
    BoxDims box{};
    int n = 0;                  // tile edge p + 1
    int64_t nelem = 0, ndof = 0, n1 = 0;
    int ness = -1;              // essential DOFs of the bound operator's box
    int step = 0;               // Adam steps taken
    // parameters and optimiser state (device FP32)
    float *params = nullptr, *grads = nullptr, *adam_m = nullptr, *adam_v = nullptr, *wt = nullptr;
    void *wpack = nullptr;      // lane-ordered FP16 weights of the MFMA inference kernel
    // operator-dependent arrays
    float *logk = nullptr;      // [nelem][P]
    double *inv_mult = nullptr; // [ndof]
    double *dinv = nullptr;     // [ndof] 1 / diag(A_c): the Jacobi term of the preconditioner
    // network activations and gradients
    float *x0 = nullptr, *s = nullptr, *a1 = nullptr, *a2 = nullptr, *out = nullptr;
    float *ga1 = nullptr, *ga2 = nullptr, *gout = nullptr, *partial = nullptr;
    // coarse level
    double *gll = nullptr, *S = nullptr, *cdinv = nullptr, *cr = nullptr, *cu = nullptr, *cz = nullptr, *cp0 = nullptr,
           *cp1 = nullptr, *cAp = nullptr, *cpart = nullptr, *ct1 = nullptr, *ct2 = nullptr;
    int32_t *cess = nullptr;
    int ncess = 0;
    CoarseScalars *csc = nullptr;
    // the fixed-iteration coarse solve as one HIP graph (kernel nodes only), rebuilt when
    // the binding or the iteration count changes
    hipStream_t cap_stream = nullptr;
    hipGraph_t cgraph = nullptr;
    hipGraphExec_t cexec = nullptr;
    int cgraph_iters = -1;
    // FP64 work vectors [ndof]
    double *v0 = nullptr, *v1 = nullptr, *v2 = nullptr, *v3 = nullptr, *red = nullptr, *dsc = nullptr;
    double *tr_r = nullptr, *tr_t = nullptr;  // training pair (allocated on first use)

    void free_graph()
    {
        if (cexec) (void)hipGraphExecDestroy(cexec);
        if (cgraph) (void)hipGraphDestroy(cgraph);
        cexec = nullptr;
        cgraph = nullptr;
        cgraph_iters = -1;
    }
    void free_bound()
    {
        free_graph();
        for (void *p : {(void *)logk, (void *)inv_mult, (void *)dinv, (void *)x0, (void *)s, (void *)a1, (void *)a2,
                        (void *)out, (void *)ga1, (void *)ga2, (void *)gout, (void *)gll, (void *)S, (void *)cdinv,
                        (void *)cr, (void *)cu, (void *)cz, (void *)cp0, (void *)cp1, (void *)cAp, (void *)cpart,
                        (void *)cess, (void *)csc, (void *)ct1, (void *)ct2, (void *)v0, (void *)v1, (void *)v2, (void *)v3,
                        (void *)tr_r, (void *)tr_t})
            dfree(p);
        logk = nullptr; inv_mult = dinv = nullptr; x0 = s = a1 = a2 = out = ga1 = ga2 = gout = nullptr;
        gll = S = cdinv = cr = cu = cz = cp0 = cp1 = cAp = cpart = ct1 = ct2 = nullptr;
        cess = nullptr; csc = nullptr; v0 = v1 = v2 = v3 = tr_r = tr_t = nullptr;
        if (coarse) pa_destroy(coarse);
        coarse = nullptr;
        op = nullptr;
    }
    ~pa_lp()
    {
        free_bound();
        if (cap_stream) (void)hipStreamDestroy(cap_stream);
        for (void *p : {(void *)params, (void *)grads, (void *)adam_m, (void *)adam_v, (void *)wt, (void *)partial,
                        (void *)red, (void *)dsc, wpack})
            dfree(p);
    }
};

namespace {

int check_opts(const pa_lp_opts *o)
{
    if (!o) return arg_error("pa_lp: opts is NULL");
    if (o->use_net != 0 && o->use_net != 1) return arg_error("pa_lp: use_net must be 0 or 1");
    if (o->use_coarse != 0 && o->use_coarse != 1) return arg_error("pa_lp: use_coarse must be 0 or 1");
    if (o->use_coarse && o->coarse_iters < 1) return arg_error("pa_lp: coarse_iters must be >= 1");
    if (o->coarse_iters > 1000) return arg_error("pa_lp: coarse_iters must be <= 1000");
    if (o->loss != PA_LP_LOSS_ENERGY && o->loss != PA_LP_LOSS_L2) return arg_error("pa_lp: unknown loss");
    if (!(o->lr >= 0.0)) return arg_error("pa_lp: lr must be >= 0");
    if (o->infer_fp16 != 0 && o->infer_fp16 != 1) return arg_error("pa_lp: infer_fp16 must be 0 or 1");
    return PA_OK;
}

// He-normal initialisation of the hidden layers (std::mt19937_64 and the standard
// library's normal distribution), zero biases and a zero output layer.
std::vector<float> default_params(int seed)
{
    std::vector<float> p(kNetParams, 0.0f);
    std::mt19937_64 g((uint64_t)seed * 0x9E3779B97F4A7C15ull + 12345u);
    std::normal_distribution<double> nd(0.0, 1.0);
    auto fill = [&](int off, int count, double fan_in, double gain) {
        const double sd = std::sqrt(gain / fan_in);
        for (int i = 0; i < count; ++i) p[off + i] = (float)(nd(g) * sd);
    };
    fill(kNetOffW1, kNetW1, 27.0 * kNetCin, 2.0);
    fill(kNetOffW2, kNetW2, 27.0 * kNetCh, 2.0);
    // the output layer starts at zero: the untrained network adds nothing to Jacobi
    return p;
}

uint64_t fnv1a(const void *data, size_t n)
{
    const unsigned char *c = (const unsigned char *)data;
    uint64_t h = 1469598103934665603ull;
    for (size_t i = 0; i < n; ++i) {
        h ^= c[i];
        h *= 1099511628211ull;
    }
    return h;
}

// Build everything that depends on the operator.
int bind(pa_lp *lp, pa_op *op, hipStream_t s)
{
    if (op->nx <= 0) return arg_error("pa_lp: the operator must be a structured box");
    if (!(op->ops & PA_DIFFUSION)) return arg_error("pa_lp: the operator must contain diffusion");
    if (op->d < 3 || op->d > 5) {
        set_error("pa_lp: the network is compiled for p = 2, 3, 4");
        return PA_ERR_UNSUPPORTED;
    }
    lp->free_bound();
    lp->op = op;
    lp->n = op->d;
    lp->nelem = op->nelem;
    lp->ndof = op->ndof;
    lp->box = BoxDims{op->nx, op->ny, op->nz, op->p};
    lp->ness = op->ness;
    const int64_t P = (int64_t)lp->n * lp->n * lp->n, ne = lp->nelem, nd = lp->ndof;
    HIP_OK(dalloc(&lp->logk, ne * P));
    HIP_OK(dalloc(&lp->inv_mult, nd));
    HIP_OK(dalloc(&lp->dinv, nd));
    // network tiles: the +r tile of every element, then the -r tile
    HIP_OK(dalloc(&lp->x0, 2 * ne * kNetCin * P));
    HIP_OK(dalloc(&lp->s, ne));
    HIP_OK(dalloc(&lp->a1, 2 * ne * kNetCh * P));
    HIP_OK(dalloc(&lp->a2, 2 * ne * kNetCh * P));
    HIP_OK(dalloc(&lp->out, 2 * ne * P));
    HIP_OK(dalloc(&lp->v0, nd));
    HIP_OK(dalloc(&lp->v1, nd));
    HIP_OK(dalloc(&lp->v2, nd));
    HIP_OK(dalloc(&lp->v3, nd));
    HIP_OK(logk_tiles(op, lp->logk, s));
    HIP_OK(nn_inv_mult(lp->n, ne, nd, op->d_elem_dofs, lp->inv_mult, s));
    int rc = pa_diag(op, lp->dinv, 1, s);
    if (rc) return rc;
    HIP_OK(vec_recip(lp->dinv, lp->dinv, nd, s));

    // coarse operator: same vertices, hexes and coefficient, order 1, 3-point Gauss
    std::vector<double> vert((size_t)op->nvert * 3);
    std::vector<int32_t> hex((size_t)op->nelem * 8);
    HIP_OK(hipMemcpy(vert.data(), op->d_vert, vert.size() * sizeof(double), hipMemcpyDeviceToHost));
    HIP_OK(hipMemcpy(hex.data(), op->d_hex, hex.size() * sizeof(int32_t), hipMemcpyDeviceToHost));
    pa_coeff_desc cd{};
    cd.kind = op->coeff.kind;
    cd.value = op->coeff.value;
    cd.amp = op->coeff.amp;
    cd.freq = op->coeff.freq;
    std::vector<double> grid;
    if (op->coeff.kind == PA_COEFF_GRID) {
        grid.resize((size_t)op->coeff.gx * op->coeff.gy * op->coeff.gz);
        HIP_OK(hipMemcpy(grid.data(), op->d_grid, grid.size() * sizeof(double), hipMemcpyDeviceToHost));
        cd.grid = grid.data();
        cd.gx = op->coeff.gx;
        cd.gy = op->coeff.gy;
        cd.gz = op->coeff.gz;
    }
    pa_mesh_desc md{};
    md.nvert = op->nvert;
    md.vert_xyz = vert.data();
    md.nelem = op->nelem;
    md.hex = hex.data();
    md.nx = op->nx;
    md.ny = op->ny;
    md.nz = op->nz;
    md.ess_mode = 0;
    rc = pa_setup(&md, 1, 3, &cd, (uint32_t)op->ops, s, &lp->coarse);
    if (rc) return rc;
    pa_op *c = lp->coarse;
    const int64_t n1 = c->ndof;
    lp->n1 = n1;
    // coarse essential DOFs: the box boundary when the fine operator constrains DOFs
    std::vector<uint8_t> ess1((size_t)n1, 0);
    std::vector<int32_t> cl;
    if (op->ness > 0) {
        const int64_t Cx = op->nx + 1, Cy = op->ny + 1, Cz = op->nz + 1;
        for (int64_t K = 0; K < Cz; ++K)
            for (int64_t J = 0; J < Cy; ++J)
                for (int64_t I = 0; I < Cx; ++I)
                    if (I == 0 || J == 0 || K == 0 || I == Cx - 1 || J == Cy - 1 || K == Cz - 1) {
                        const int64_t i = I + Cx * (J + Cy * K);
                        ess1[(size_t)i] = 1;
                        cl.push_back((int32_t)i);
                    }
    }
    lp->ncess = (int)cl.size();
    uint8_t *d_ess1 = nullptr;
    HIP_OK(dalloc(&d_ess1, (size_t)n1));
    std::unique_ptr<void, void (*)(void *)> g1(d_ess1, dfree);
    HIP_OK(hipMemcpy(d_ess1, ess1.data(), (size_t)n1, hipMemcpyHostToDevice));
    if (!cl.empty()) {
        HIP_OK(dalloc(&lp->cess, cl.size()));
        HIP_OK(hipMemcpy(lp->cess, cl.data(), cl.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    HIP_OK(dalloc(&lp->S, 27 * n1));
    HIP_OK(dalloc(&lp->cdinv, n1));
    HIP_OK(dalloc(&lp->cr, n1));
    HIP_OK(dalloc(&lp->cu, n1));
    HIP_OK(dalloc(&lp->cz, n1));
    HIP_OK(dalloc(&lp->cp0, n1));
    HIP_OK(dalloc(&lp->cp1, n1));
    HIP_OK(dalloc(&lp->cAp, n1));
    HIP_OK(dalloc(&lp->cpart, (n1 + 255) / 256));  // one partial per coarse block (256 threads)
    HIP_OK(dalloc(&lp->csc, 1));
    {
        const int64_t My = (int64_t)op->ny * op->p + 1, Mz = (int64_t)op->nz * op->p + 1;
        HIP_OK(dalloc(&lp->ct1, (size_t)(op->nx + 1) * My * Mz));
        HIP_OK(dalloc(&lp->ct2, (size_t)(op->nx + 1) * (op->ny + 1) * Mz));
    }
    HIP_OK(hipMemset(lp->csc, 0, sizeof(CoarseScalars)));
    HIP_OK(dalloc(&lp->gll, (size_t)op->d));
    HIP_OK(hipMemcpy(lp->gll, op->tab.nodes.data(), (size_t)op->d * sizeof(double), hipMemcpyHostToDevice));
    // 27-point stencil of the constrained coarse operator by probing with 27 class vectors
    for (int cls = 0; cls < 27; ++cls) {
        HIP_OK(coarse_probe_vec(lp->box, cls, lp->cr, s));
        rc = do_apply(c, c->variant, lp->cr, lp->cu, s);
        if (rc) return rc;
        HIP_OK(coarse_probe_gather(lp->box, cls, lp->cu, d_ess1, lp->S, s));
    }
    HIP_OK(coarse_dinv(n1, lp->S, lp->cdinv, s));
    HIP_OK(hipStreamSynchronize(s));
    return PA_OK;
}

int ensure_training(pa_lp *lp)
{
    const int64_t P = (int64_t)lp->n * lp->n * lp->n;
    if (!lp->ga1) HIP_OK(dalloc(&lp->ga1, 2 * lp->nelem * kNetCh * P));
    if (!lp->ga2) HIP_OK(dalloc(&lp->ga2, 2 * lp->nelem * kNetCh * P));
    if (!lp->gout) HIP_OK(dalloc(&lp->gout, 2 * lp->nelem * P));
    if (!lp->partial) HIP_OK(dalloc(&lp->partial, (size_t)nn_partial_floats()));
    if (!lp->tr_r) HIP_OK(dalloc(&lp->tr_r, lp->ndof));
    if (!lp->tr_t) HIP_OK(dalloc(&lp->tr_t, lp->ndof));
    return PA_OK;
}

// z (+)= W G^T (s_e NN(x0_e)), then zero on the essential DOFs.  The FP32 path keeps the
// activations for the backward pass; the FP16 path is the fused inference kernel.
int net_part(pa_lp *lp, const double *r, double *z, hipStream_t s, bool fp16, bool accumulate = false,
             double scale = 1.0)
{
    pa_op *op = lp->op;
    if (!accumulate) HIP_OK(vec_fill(z, 0.0, lp->ndof, s));
    if (fp16) {
        HIP_OK(nn_infer16(lp->n, lp->nelem, lp->params, lp->wpack, r, op->d_elem_dofs, lp->logk, lp->inv_mult, scale,
                          z, s));
    } else {
        HIP_OK(nn_input(lp->n, lp->nelem, r, op->d_elem_dofs, lp->logk, lp->x0, lp->s, s));
        HIP_OK(nn_forward(lp->n, 2 * lp->nelem, lp->params, lp->wt, lp->x0, lp->a1, lp->a2, lp->out, s));
        HIP_OK(nn_output(lp->n, lp->nelem, lp->out, lp->s, op->d_elem_dofs, lp->inv_mult, scale, z, s));
    }
    if (op->ness) HIP_OK(vec_zero_list(z, op->d_ess, op->ness, s));
    return PA_OK;
}

// Capture the coarse Jacobi-PCG (2 kernels per iteration) into a graph so that one
// launch replaces 2k + 1; the kernels clear what they need themselves (no memset nodes).
int ensure_coarse_graph(pa_lp *lp)
{
    if (lp->cexec && lp->cgraph_iters == lp->o.coarse_iters) return PA_OK;
    lp->free_graph();
    if (!lp->cap_stream) HIP_OK(hipStreamCreateWithFlags(&lp->cap_stream, hipStreamNonBlocking));
    HIP_OK(hipStreamBeginCapture(lp->cap_stream, hipStreamCaptureModeThreadLocal));
    const hipError_t e1 = coarse_pcg(lp->box, lp->S, lp->cdinv, lp->cr, lp->cu, lp->cz, lp->cp0, lp->cp1, lp->cAp,
                                     lp->cpart, lp->csc, lp->o.coarse_iters, lp->cap_stream);
    const hipError_t e2 = hipStreamEndCapture(lp->cap_stream, &lp->cgraph);
    HIP_OK(e1);
    HIP_OK(e2);
    HIP_OK(hipGraphInstantiate(&lp->cexec, lp->cgraph, nullptr, nullptr, 0));
    lp->cgraph_iters = lp->o.coarse_iters;
    return PA_OK;
}

// z (+)= P1 A1^{-1} P1^T r
int coarse_part(pa_lp *lp, const double *r, double *z, bool add, hipStream_t s)
{
    HIP_OK(coarse_restrict(lp->box, lp->gll, r, lp->cr, lp->ct1, lp->ct2, s));
    if (lp->ncess) HIP_OK(vec_zero_list(lp->cr, lp->cess, lp->ncess, s));
    int rc = ensure_coarse_graph(lp);
    if (rc) return rc;
    HIP_OK(hipGraphLaunch(lp->cexec, s));
    HIP_OK(coarse_prolong(lp->box, lp->gll, lp->cu, z, add, s));
    if (lp->op->ness) HIP_OK(vec_zero_list(z, lp->op->d_ess, lp->op->ness, s));
    return PA_OK;
}

// loss and gradient of the network part against t; grads accumulate into lp->grads
// (zeroed first).  The loss value is left in lp->dsc[2].
int loss_grad(pa_lp *lp, const double *r, const double *t, hipStream_t s)
{
    int rc = ensure_training(lp);
    if (rc) return rc;
    pa_op *op = lp->op;
    const int64_t nd = lp->ndof;
    double *z = lp->v0, *diff = lp->v1, *gz = lp->v2, *At = lp->v3;
    rc = net_part(lp, r, z, s, false);
    if (rc) return rc;
    HIP_OK(vec_sub(diff, z, t, nd, s));  // zero on essential DOFs: z and t both vanish there
    if (lp->o.loss == PA_LP_LOSS_ENERGY) {
        rc = do_apply_constrained(op, diff, gz, s);
        if (rc) return rc;
        rc = do_apply_constrained(op, t, At, s);
        if (rc) return rc;
        HIP_OK(vec_dot<double>(diff, gz, nd, lp->red, lp->dsc + 0, s));
        HIP_OK(vec_dot<double>(t, At, nd, lp->red, lp->dsc + 1, s));
    } else {
        HIP_OK(vec_copy(gz, diff, nd, s));
        HIP_OK(vec_dot<double>(diff, diff, nd, lp->red, lp->dsc + 0, s));
        HIP_OK(vec_dot<double>(t, t, nd, lp->red, lp->dsc + 1, s));
    }
    // gz <- 2 gz / den, L = num / den (device scalars)
    HIP_OK(vec_loss_scale(gz, nd, lp->dsc, s));
    if (op->ness) HIP_OK(vec_zero_list(gz, op->d_ess, op->ness, s));
    HIP_OK(nn_output_grad(lp->n, lp->nelem, gz, lp->s, op->d_elem_dofs, lp->inv_mult, lp->gout, s));
    HIP_OK(vec_fill_f32(lp->grads, 0.0f, kNetParams, s));
    HIP_OK(nn_backward(lp->n, 2 * lp->nelem, lp->params, lp->x0, lp->a1, lp->a2, lp->gout, lp->ga2, lp->ga1,
                       lp->grads, lp->wt, lp->partial, s));
    return PA_OK;
}

}  // namespace

extern "C" int pa_lp_num_params(void) { return kNetParams; }

extern "C" int pa_lp_create(pa_op *op, const pa_lp_opts *o, pa_lp **out)
{
    PA_TRY
    if (!out) return arg_error("pa_lp_create: out is NULL");
    *out = nullptr;
    if (!op) return arg_error("pa_lp_create: op is NULL");
    int rc = check_opts(o);
    if (rc) return rc;
    std::unique_ptr<pa_lp> lp(new pa_lp);
    lp->o = *o;
    HIP_OK(hipSetDevice(op->device));
    HIP_OK(dalloc(&lp->params, kNetParams));
    HIP_OK(dalloc(&lp->grads, kNetParams));
    HIP_OK(dalloc(&lp->adam_m, kNetParams));
    HIP_OK(dalloc(&lp->adam_v, kNetParams));
    HIP_OK(dalloc(&lp->wt, kNetW1 + kNetW2 + kNetW3));
    HIP_OK(dalloc(&lp->red, 2 * kRedBlocks));
    HIP_OK(dalloc(&lp->dsc, 4));
    HIP_OK(hipMalloc(&lp->wpack, (size_t)nn_pack16_bytes()));
    const std::vector<float> p0 = default_params(o->seed);
    HIP_OK(hipMemcpy(lp->params, p0.data(), kNetParams * sizeof(float), hipMemcpyHostToDevice));
    HIP_OK(hipMemset(lp->grads, 0, kNetParams * sizeof(float)));
    HIP_OK(hipMemset(lp->adam_m, 0, kNetParams * sizeof(float)));
    HIP_OK(hipMemset(lp->adam_v, 0, kNetParams * sizeof(float)));
    rc = bind(lp.get(), op, nullptr);
    if (rc) return rc;
    *out = lp.release();
    return PA_OK;
    PA_CATCH
}

extern "C" int pa_lp_bind(pa_lp *lp, pa_op *op)
{
    PA_TRY
    if (!lp || !op) return arg_error("pa_lp_bind: NULL argument");
    if (lp->ness >= 0 && (op->nx != lp->box.nx || op->ny != lp->box.ny || op->nz != lp->box.nz ||
                          op->p != lp->box.p || op->ness != lp->ness))
        return arg_error("pa_lp_bind: the operator's box, order or essential DOFs differ");
    return bind(lp, op, nullptr);
    PA_CATCH
}

extern "C" int pa_lp_configure(pa_lp *lp, const pa_lp_opts *o)
{
    if (!lp) return arg_error("pa_lp_configure: lp is NULL");
    int rc = check_opts(o);
    if (rc) return rc;
    const int seed = lp->o.seed;
    lp->o = *o;
    lp->o.seed = seed;
    return PA_OK;
}

extern "C" int pa_lp_get_params(pa_lp *lp, float *host, int n)
{
    if (!lp || !host || n != kNetParams) return arg_error("pa_lp_get_params: NULL argument or wrong count");
    HIP_OK(hipMemcpy(host, lp->params, kNetParams * sizeof(float), hipMemcpyDeviceToHost));
    return PA_OK;
}

extern "C" int pa_lp_set_params(pa_lp *lp, const float *host, int n)
{
    if (!lp || !host || n != kNetParams) return arg_error("pa_lp_set_params: NULL argument or wrong count");
    for (int i = 0; i < n; ++i)
        if (!std::isfinite(host[i])) return arg_error("pa_lp_set_params: non-finite parameter");
    HIP_OK(hipMemcpy(lp->params, host, kNetParams * sizeof(float), hipMemcpyHostToDevice));
    HIP_OK(hipMemset(lp->adam_m, 0, kNetParams * sizeof(float)));
    HIP_OK(hipMemset(lp->adam_v, 0, kNetParams * sizeof(float)));
    lp->step = 0;
    return PA_OK;
}

extern "C" int pa_lp_logk(pa_lp *lp, float *dev_out)
{
    if (!lp || !dev_out) return arg_error("pa_lp_logk: NULL argument");
    const int64_t P = (int64_t)lp->n * lp->n * lp->n;
    HIP_OK(hipMemcpy(dev_out, lp->logk, lp->nelem * P * sizeof(float), hipMemcpyDeviceToDevice));
    return PA_OK;
}

int hexpa::lp_precondition(pa_lp *lp, const double *r, double *z, hipStream_t s)
{
    // Jacobi, plus the network's learned correction
    HIP_OK(vec_mul(z, lp->dinv, r, lp->ndof, s));
    if (lp->o.use_net) {
        int rc = net_part(lp, r, z, s, lp->o.infer_fp16 != 0, true, lp->o.net_scale > 0.0 ? lp->o.net_scale : 1.0);
        if (rc) return rc;
    }
    if (lp->o.use_coarse) {
        int rc = coarse_part(lp, r, z, true, s);
        if (rc) return rc;
    } else if (lp->op->ness) {
        HIP_OK(vec_zero_list(z, lp->op->d_ess, lp->op->ness, s));
    }
    return PA_OK;
}

pa_op *hexpa::lp_operator(const pa_lp *lp) { return lp->op; }

extern "C" int pa_lp_apply(pa_lp *lp, const double *r, double *z, void *stream)
{
    PA_TRY
    if (!lp || !r || !z) return arg_error("pa_lp_apply: NULL argument");
    return lp_precondition(lp, r, z, as_stream(stream));
    PA_CATCH
}

extern "C" int pa_lp_coarse(pa_lp *lp, const double *r, double *z, void *stream)
{
    PA_TRY
    if (!lp || !r || !z) return arg_error("pa_lp_coarse: NULL argument");
    if (lp->o.coarse_iters < 1) return arg_error("pa_lp_coarse: coarse_iters must be >= 1");
    return coarse_part(lp, r, z, false, as_stream(stream));
    PA_CATCH
}

extern "C" int pa_lp_net(pa_lp *lp, const double *r, double *z, void *stream)
{
    PA_TRY
    if (!lp || !r || !z) return arg_error("pa_lp_net: NULL argument");
    return net_part(lp, r, z, as_stream(stream), lp->o.infer_fp16 != 0);
    PA_CATCH
}

extern "C" int pa_lp_loss_grad(pa_lp *lp, const double *r, const double *t, double *loss, float *grad_host,
                               void *stream)
{
    PA_TRY
    if (!lp || !r || !t || !loss) return arg_error("pa_lp_loss_grad: NULL argument");
    hipStream_t s = as_stream(stream);
    int rc = loss_grad(lp, r, t, s);
    if (rc) return rc;
    HIP_OK(hipMemcpyAsync(loss, lp->dsc + 2, sizeof(double), hipMemcpyDeviceToHost, s));
    if (grad_host) HIP_OK(hipMemcpyAsync(grad_host, lp->grads, kNetParams * sizeof(float), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    return PA_OK;
    PA_CATCH
}

extern "C" int pa_lp_train_step(pa_lp *lp, const double *b, const double *xstar, const double *xk, double *loss,
                                void *stream)
{
    PA_TRY
    if (!lp || !b || !xstar || !xk) return arg_error("pa_lp_train_step: NULL argument");
    hipStream_t s = as_stream(stream);
    int rc = ensure_training(lp);
    if (rc) return rc;
    const int64_t nd = lp->ndof;
    double *rbuf = lp->tr_r, *tbuf = lp->tr_t;
    rc = do_apply_constrained(lp->op, xk, rbuf, s);
    if (rc) return rc;
    HIP_OK(vec_sub(rbuf, b, rbuf, nd, s));
    HIP_OK(vec_sub(tbuf, xstar, xk, nd, s));
    // the network learns what Jacobi and the coarse correction leave of the error
    HIP_OK(vec_mul(lp->v0, lp->dinv, rbuf, nd, s));
    HIP_OK(vec_sub(tbuf, tbuf, lp->v0, nd, s));
    if (lp->o.use_coarse) {
        rc = coarse_part(lp, rbuf, lp->v0, false, s);
        if (rc) return rc;
        HIP_OK(vec_sub(tbuf, tbuf, lp->v0, nd, s));
    }
    if (lp->op->ness) HIP_OK(vec_zero_list(tbuf, lp->op->d_ess, lp->op->ness, s));
    rc = loss_grad(lp, rbuf, tbuf, s);
    if (rc) return rc;
    lp->step += 1;
    HIP_OK(nn_adam(lp->params, lp->grads, lp->adam_m, lp->adam_v, kNetParams, lp->o.lr, lp->step, s));
    if (loss) {
        HIP_OK(hipMemcpyAsync(loss, lp->dsc + 2, sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
    }
    return PA_OK;
    PA_CATCH
}

namespace {
// splitmix64 (Steele, Lea & Flood 2014): the pair order of each (epoch, draw) is a
// Fisher-Yates shuffle driven by this counter-based generator
uint64_t splitmix64(uint64_t &state)
{
    uint64_t z = (state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
}  // namespace

extern "C" int pa_lp_train(pa_lp *lp, const pa_train_set *set, pa_train_log *log, void *stream)
{
    PA_TRY
    if (!lp || !set || !log) return arg_error("pa_lp_train: NULL argument");
    if (set->ndraws < 0 || (set->ndraws > 0 && (!set->ops || !set->xstar)))
        return arg_error("pa_lp_train: ndraws < 0, or ops / xstar missing");
    if (set->capture != PA_LP_CAPTURE_FCG && set->capture != PA_LP_CAPTURE_JACOBI)
        return arg_error("pa_lp_train: unknown capture mode");
    if (set->n_capture < 1 || !set->capture_at) return arg_error("pa_lp_train: need n_capture >= 1 and capture_at");
    for (int j = 0; j < set->n_capture; ++j)
        if (set->capture_at[j] < 0 || (j > 0 && set->capture_at[j] <= set->capture_at[j - 1]))
            return arg_error("pa_lp_train: capture_at must be ascending and >= 0");
    if (set->epochs < 1) return arg_error("pa_lp_train: epochs must be >= 1");
    if (log->max_steps < 0 || (log->max_steps > 0 && !log->loss))
        return arg_error("pa_lp_train: log->loss is NULL with max_steps > 0");
    for (int d = 0; d < set->ndraws; ++d)
        if (!set->ops[d] || !set->xstar[d]) return arg_error("pa_lp_train: NULL operator or solution");
    log->steps = 0;
    log->seconds_capture = log->seconds_train = 0.0;
    if (set->ndraws == 0) return PA_OK;
    hipStream_t s = as_stream(stream);
    const int64_t nd = set->ops[0]->ndof;
    const int ncap = set->n_capture;
    double *b = nullptr, *x = nullptr, *cap = nullptr;
    HIP_OK(dalloc(&b, (size_t)nd));
    std::unique_ptr<void, void (*)(void *)> g1(b, dfree);
    HIP_OK(dalloc(&x, (size_t)nd));
    std::unique_ptr<void, void (*)(void *)> g2(x, dfree);
    HIP_OK(dalloc(&cap, (size_t)nd * ncap));
    std::unique_ptr<void, void (*)(void *)> g3(cap, dfree);
    std::vector<int> order;
    for (int ep = 0; ep < set->epochs; ++ep) {
        for (int d = 0; d < set->ndraws; ++d) {
            pa_op *op = set->ops[d];
            if (op->ndof != nd) return arg_error("pa_lp_train: the operators differ in size");
            auto t0 = std::chrono::steady_clock::now();
            int rc = (lp->op == op) ? PA_OK : pa_lp_bind(lp, op);
            if (rc) return rc;
            // b = A_c x*, then the iterates of the capture solve from x = 0
            rc = do_apply_constrained(op, set->xstar[d], b, s);
            if (rc) return rc;
            HIP_OK(vec_fill(x, 0.0, nd, s));
            pa_cg_opts o;
            std::memset(&o, 0, sizeof(o));
            o.rtol = 1e-10;
            o.max_it = set->capture_at[ncap - 1] + 1;
            o.mode = set->capture == PA_LP_CAPTURE_FCG ? PA_CG_FCG : PA_CG_JACOBI;
            o.check_every = 8;
            o.constrained = 1;
            o.lp = set->capture == PA_LP_CAPTURE_FCG ? lp : nullptr;
            o.n_capture = ncap;
            o.capture_at = set->capture_at;
            o.capture_x = cap;
            pa_cg_result res;
            rc = cg_solve(op, b, x, &o, &res, stream);
            if (rc != PA_OK && rc != PA_ERR_NOT_CONVERGED) return rc;
            int reached = 0;
            while (reached < ncap && set->capture_at[reached] <= res.iters) ++reached;
            auto t1 = std::chrono::steady_clock::now();
            // one training step per captured pair, in a seeded random order
            order.resize(reached);
            for (int j = 0; j < reached; ++j) order[j] = j;
            uint64_t st = ((uint64_t)set->seed << 32) ^ ((uint64_t)ep << 20) ^ (uint64_t)d;
            for (int j = reached - 1; j > 0; --j) std::swap(order[j], order[(int)(splitmix64(st) % (uint64_t)(j + 1))]);
            for (int j : order) {
                double L = 0.0;
                const bool keep = log->steps < log->max_steps;
                rc = pa_lp_train_step(lp, b, set->xstar[d], cap + (size_t)j * nd, keep ? &L : nullptr, stream);
                if (rc) return rc;
                if (keep) log->loss[log->steps] = L;
                log->steps += 1;
            }
            HIP_OK(hipStreamSynchronize(s));
            auto t2 = std::chrono::steady_clock::now();
            log->seconds_capture += std::chrono::duration<double>(t1 - t0).count();
            log->seconds_train += std::chrono::duration<double>(t2 - t1).count();
        }
    }
    return PA_OK;
    PA_CATCH
}

extern "C" int pa_lp_save(pa_lp *lp, const char *path)
{
    PA_TRY
    if (!lp || !path) return arg_error("pa_lp_save: NULL argument");
    std::vector<float> p(kNetParams);
    HIP_OK(hipMemcpy(p.data(), lp->params, kNetParams * sizeof(float), hipMemcpyDeviceToHost));
    FILE *f = std::fopen(path, "wb");
    if (!f) {
        set_error("pa_lp_save: cannot open file for writing");
        return PA_ERR_IO;
    }
    const int32_t hdr[2] = {1, kNetParams};
    const uint64_t h = fnv1a(p.data(), p.size() * sizeof(float));
    bool ok = std::fwrite("HEXPALP1", 1, 8, f) == 8 && std::fwrite(hdr, sizeof(hdr), 1, f) == 1 &&
              std::fwrite(p.data(), sizeof(float), p.size(), f) == p.size() && std::fwrite(&h, sizeof(h), 1, f) == 1;
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) {
        set_error("pa_lp_save: write failed");
        return PA_ERR_IO;
    }
    return PA_OK;
    PA_CATCH
}

extern "C" int pa_lp_load(pa_lp *lp, const char *path)
{
    PA_TRY
    if (!lp || !path) return arg_error("pa_lp_load: NULL argument");
    FILE *f = std::fopen(path, "rb");
    if (!f) {
        set_error("pa_lp_load: cannot open file");
        return PA_ERR_IO;
    }
    char magic[8];
    int32_t hdr[2];
    std::vector<float> p(kNetParams);
    uint64_t h = 0;
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "HEXPALP1", 8) == 0 &&
              std::fread(hdr, sizeof(hdr), 1, f) == 1 && hdr[0] == 1 && hdr[1] == kNetParams &&
              std::fread(p.data(), sizeof(float), p.size(), f) == p.size() && std::fread(&h, sizeof(h), 1, f) == 1 &&
              h == fnv1a(p.data(), p.size() * sizeof(float));
    std::fclose(f);
    if (!ok) {
        set_error("pa_lp_load: not a parameter file of this network (magic, version, count or checksum)");
        return PA_ERR_IO;
    }
    return pa_lp_set_params(lp, p.data(), kNetParams);
    PA_CATCH
}

extern "C" void pa_lp_destroy(pa_lp *lp) { delete lp; }
