// C-ABI of the mixed H1 x L2 operator: setup (DOF map, 1-D tables of both spaces, the
// quadrature-point data E_cm = w adj(J)_mc), the fused apply of both off-diagonal blocks,
// the lumped masses and the RK4 time stepper.
#include <cmath>
#include <cstring>
#include <memory>
#include <string>
#include <vector>

#include "capi_util.h"
#include "k_vec.h"
#include "mixed.h"

using namespace hexpa;

namespace {

void fill_dev_tables(const Tables1D &t, DevTables &ht)
{
    std::memset(&ht, 0, sizeof(ht));
    for (int a = 0; a < t.q; ++a) {
        ht.w[a] = t.qwts[a];
        ht.x[a] = t.qpts[a];
        for (int i = 0; i < t.d; ++i) {
            ht.B[a * t.d + i] = t.B[(size_t)a * t.d + i];
            ht.G[a * t.d + i] = t.G[(size_t)a * t.d + i];
        }
    }
    for (int i = 0; i < t.d; ++i) ht.nodes[i] = t.nodes[i];
}

// inverse lumped masses, made on first use of the time stepper
int ensure_minv(pa_mixed *m, hipStream_t s)
{
    if (m->d_minv_u) return PA_OK;
    const int nu = (m->pu + 1) * (m->pu + 1) * (m->pu + 1);
    double *mu = nullptr;
    HIP_OK(dalloc(&mu, (size_t)m->nelem * nu));
    std::unique_ptr<void, void (*)(void *)> g(mu, dfree);
    HIP_OK(dalloc(&m->d_minv_u, (size_t)m->nvel));
    HIP_OK(dalloc(&m->d_minv_p, (size_t)m->ndof));
    HIP_OK(vec_fill(m->d_minv_p, 0.0, m->ndof, s));
    HIP_OK(launch_mixed_lumped(m, mu, m->d_minv_p, s));
    HIP_OK(vec_recip(m->d_minv_p, m->d_minv_p, m->ndof, s));
    // the velocity mass row of node J is the same for the three components
    std::vector<double> h((size_t)m->nelem * nu), hu((size_t)m->nvel);
    HIP_OK(hipMemcpyAsync(h.data(), mu, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    for (int64_t e = 0; e < m->nelem; ++e)
        for (int c = 0; c < 3; ++c)
            for (int J = 0; J < nu; ++J) hu[(size_t)(e * 3 + c) * nu + J] = 1.0 / h[(size_t)e * nu + J];
    HIP_OK(hipMemcpy(m->d_minv_u, hu.data(), hu.size() * sizeof(double), hipMemcpyHostToDevice));
    return PA_OK;
}

}  // namespace

extern "C" void pa_mixed_destroy(pa_mixed *m)
{
    if (!m) return;
    dfree(m->d_emap);
    dfree(m->d_qdata);
    dfree(m->d_vert);
    dfree(m->d_hex);
    dfree(m->d_tabp);
    dfree(m->d_tabu);
    dfree(m->d_minv_u);
    dfree(m->d_minv_p);
    dfree(m->d_rk);
    delete m;
}

extern "C" int pa_mixed_setup(const pa_mesh_desc *mesh, const pa_mixed_desc *desc, void *stream, pa_mixed **out)
{
    PA_TRY
    if (!out) return arg_error("pa_mixed_setup: out is NULL");
    *out = nullptr;
    if (!mesh || !desc || !mesh->vert_xyz || !mesh->hex || mesh->nvert <= 0 || mesh->nelem <= 0)
        return arg_error("pa_mixed_setup: mesh or descriptor incomplete");
    if (!mixed_supported(desc->p, desc->pu, desc->q1d)) {
        set_error("pa_mixed_setup: (p, pu, q1d) must be (4, 3, 5) or (2, 1, 3)");
        return PA_ERR_UNSUPPORTED;
    }
    if (!(desc->rho > 0.0) || !(desc->bulk > 0.0)) return arg_error("pa_mixed_setup: rho and bulk must be > 0");
    if (mesh->nx <= 0 || mesh->ny <= 0 || mesh->nz <= 0 ||
        (int64_t)mesh->nx * mesh->ny * mesh->nz != mesh->nelem)
        return arg_error("pa_mixed_setup: needs a structured box (nx*ny*nz == nelem)");
    hipStream_t s = as_stream(stream);
    std::unique_ptr<pa_mixed, void (*)(pa_mixed *)> m(new pa_mixed, pa_mixed_destroy);
    m->p = desc->p; m->pu = desc->pu; m->q = desc->q1d;
    m->rho = desc->rho; m->bulk = desc->bulk;
    m->nelem = mesh->nelem; m->nvert = mesh->nvert;
    const int p = m->p, d = p + 1, d3 = d * d * d, du = m->pu + 1;
    const int64_t nx = mesh->nx, ny = mesh->ny, nz = mesh->nz, nel = mesh->nelem;
    const int64_t Mx = nx * p + 1, My = ny * p + 1, Mz = nz * p + 1;
    if (Mx * My * Mz > INT32_MAX || nel * 3 * du * du * du > INT32_MAX)
        return arg_error("pa_mixed_setup: too many DOFs for int32 indices");
    m->ndof = (int)(Mx * My * Mz);
    m->nvel = (int)(nel * 3 * du * du * du);
    for (int32_t h : std::vector<int32_t>(mesh->hex, mesh->hex + 8 * nel))
        if (h < 0 || h >= mesh->nvert) return arg_error("pa_mixed_setup: hex vertex index out of range");
    // pressure DOF map on the (n p + 1)^3 lattice (the same numbering as pa_setup)
    std::vector<int32_t> ed((size_t)nel * d3);
    for (int64_t e = 0; e < nel; ++e) {
        const int64_t ex = e % nx, ey = (e / nx) % ny, ez = e / (nx * ny);
        for (int k = 0; k < d; ++k)
            for (int j = 0; j < d; ++j)
                for (int i = 0; i < d; ++i)
                    ed[(size_t)e * d3 + i + d * (j + d * k)] =
                        (int32_t)((ex * p + i) + Mx * ((ey * p + j) + My * (ez * p + k)));
    }
    Tables1D tp, tu;
    std::string terr;
    if (!make_tables(p, m->q, tp, terr) || !make_l2_tables(m->pu, m->q, tu, terr)) return arg_error(terr.c_str());
    DevTables hp, hu;
    fill_dev_tables(tp, hp);
    fill_dev_tables(tu, hu);
    const int q3 = m->q * m->q * m->q;
    HIP_OK(hipGetDevice(&m->device));
    HIP_OK(dalloc(&m->d_emap, ed.size()));
    HIP_OK(dalloc(&m->d_qdata, (size_t)nel * 9 * q3));
    HIP_OK(dalloc(&m->d_vert, (size_t)mesh->nvert * 3));
    HIP_OK(dalloc(&m->d_hex, (size_t)nel * 8));
    HIP_OK(dalloc(&m->d_tabp, 1));
    HIP_OK(dalloc(&m->d_tabu, 1));
    HIP_OK(hipMemcpy(m->d_emap, ed.data(), ed.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(m->d_vert, mesh->vert_xyz, (size_t)mesh->nvert * 3 * sizeof(double), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(m->d_hex, mesh->hex, (size_t)nel * 8 * sizeof(int32_t), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(m->d_tabp, &hp, sizeof(hp), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(m->d_tabu, &hu, sizeof(hu), hipMemcpyHostToDevice));
    int *d_bad = nullptr;
    HIP_OK(hipMalloc((void **)&d_bad, sizeof(int)));
    std::unique_ptr<void, void (*)(void *)> gb(d_bad, dfree);
    HIP_OK(hipMemsetAsync(d_bad, 0, sizeof(int), s));
    HIP_OK(launch_mixed_qdata(m.get(), d_bad, s));
    int bad = 0;
    HIP_OK(hipMemcpyAsync(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (bad) {
        set_error("pa_mixed_setup: an element has det J <= 0 at a quadrature point");
        return PA_ERR_MESH;
    }
    *out = m.release();
    return PA_OK;
    PA_CATCH
}

extern "C" int pa_mixed_apply(pa_mixed *m, const double *u, const double *p, double *yu, double *yp, void *stream)
{
    PA_TRY
    if (!m || !u || !p || !yu || !yp) return arg_error("pa_mixed_apply: NULL argument");
    if ((const void *)u == (const void *)yu || (const void *)p == (const void *)yp || (const void *)u == (const void *)yp ||
        (const void *)p == (const void *)yu)
        return arg_error("pa_mixed_apply: outputs must not alias inputs");
    hipStream_t s = as_stream(stream);
    HIP_OK(vec_fill(yp, 0.0, m->ndof, s));
    HIP_OK(launch_mixed(m, u, p, yu, yp, s));
    return PA_OK;
    PA_CATCH
}

extern "C" int pa_mixed_lumped(pa_mixed *m, double *mu, double *mp, void *stream)
{
    PA_TRY
    if (!m || !mu || !mp) return arg_error("pa_mixed_lumped: NULL argument");
    hipStream_t s = as_stream(stream);
    HIP_OK(vec_fill(mp, 0.0, m->ndof, s));
    HIP_OK(launch_mixed_lumped(m, mu, mp, s));
    return PA_OK;
    PA_CATCH
}

extern "C" int pa_mixed_rk4(pa_mixed *m, double *u, double *p, double dt, int nsteps, void *stream)
{
    PA_TRY
    if (!m || !u || !p) return arg_error("pa_mixed_rk4: NULL argument");
    if (nsteps < 0 || !std::isfinite(dt)) return arg_error("pa_mixed_rk4: need nsteps >= 0 and a finite dt");
    hipStream_t s = as_stream(stream);
    int rc = ensure_minv(m, s);
    if (rc) return rc;
    const int64_t nv = m->nvel, np = m->ndof;
    if (!m->d_rk) HIP_OK(dalloc(&m->d_rk, (size_t)(3 * nv + 3 * np)));
    double *yu = m->d_rk, *au = yu + nv, *xu = au + nv;
    double *yp = xu + nv, *ap = yp + np, *xp = ap + np;
    // x' = f(x) with f(u, p) = (-Mu^{-1} G p, -Mp^{-1} (-G^T u)): each stage is one fused
    // apply and one combination kernel per field
    const double cs[4] = {0.5 * dt, 0.5 * dt, dt, dt / 6.0};  // next stage offset / final weight
    const double ca[4] = {0.0, 2.0, 2.0, 1.0};                // weight of k in the accumulator
    for (int n = 0; n < nsteps; ++n) {
        for (int st = 0; st < 4; ++st) {
            const double *su = st == 0 ? u : xu;
            const double *sp = st == 0 ? p : xp;
            HIP_OK(vec_fill(yp, 0.0, np, s));
            HIP_OK(launch_mixed(m, su, sp, yu, yp, s));
            const int first = st == 0, last = st == 3;
            HIP_OK(launch_rk_stage(nv, yu, m->d_minv_u, u, au, xu, first, ca[st], cs[st], last, s));
            HIP_OK(launch_rk_stage(np, yp, m->d_minv_p, p, ap, xp, first, ca[st], cs[st], last, s));
        }
    }
    return PA_OK;
    PA_CATCH
}

extern "C" int pa_mixed_set_grid_cap(pa_mixed *m, int max_workgroups)
{
    if (!m) return arg_error("pa_mixed_set_grid_cap: NULL handle");
    if (max_workgroups < 0) return arg_error("pa_mixed_set_grid_cap: max_workgroups must be >= 0");
    m->grid_cap = max_workgroups;
    return PA_OK;
}

extern "C" int pa_mixed_info(const pa_mixed *m, pa_mixed_info_t *info)
{
    if (!m || !info) return arg_error("pa_mixed_info: NULL argument");
    info->p = m->p; info->pu = m->pu; info->q1d = m->q;
    info->nelem = m->nelem; info->ndof_p = m->ndof; info->ndof_u = m->nvel;
    info->elems_per_block = mixed_elems_per_group(m->p, m->pu, m->q);
    info->qdata_bytes = (int64_t)m->nelem * 9 * m->q * m->q * m->q * 8;
    return PA_OK;
}
