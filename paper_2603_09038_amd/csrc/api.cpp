// C-ABI of the hexpa library: operator setup/apply/diag/load, Jacobi-PCG, diagnostics.
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "capi_util.h"
#include "internal.h"
#include "k_vec.h"

namespace hexpa {

static thread_local std::string g_err;
void set_error(const std::string &msg) { g_err = msg; }

hipError_t launch_apply_p1(const pa_op *, int, const double *, double *, const int32_t *, int, double *, hipStream_t,
                           bool *);
hipError_t launch_apply_p2(const pa_op *, int, const double *, double *, const int32_t *, int, double *, hipStream_t,
                           bool *);
hipError_t launch_apply_p3(const pa_op *, int, const double *, double *, const int32_t *, int, double *, hipStream_t,
                           bool *);
hipError_t launch_apply_p4(const pa_op *, int, const double *, double *, const int32_t *, int, double *, hipStream_t,
                           bool *);
hipError_t launch_apply_p5(const pa_op *, int, const double *, double *, const int32_t *, int, double *, hipStream_t,
                           bool *);
hipError_t launch_apply_p6(const pa_op *, int, const double *, double *, const int32_t *, int, double *, hipStream_t,
                           bool *);
hipError_t launch_apply_p7(const pa_op *, int, const double *, double *, const int32_t *, int, double *, hipStream_t,
                           bool *);
hipError_t launch_apply_p8(const pa_op *, int, const double *, double *, const int32_t *, int, double *, hipStream_t,
                           bool *);

hipError_t launch_apply(const pa_op *op, int variant, const double *x, double *y, const int32_t *elist, int n,
                        hipStream_t s, bool *ok, double *qbuf)
{
    if (!qbuf) qbuf = op->d_qbuf;
    switch (op->p) {
    case 1: return launch_apply_p1(op, variant, x, y, elist, n, qbuf, s, ok);
    case 2: return launch_apply_p2(op, variant, x, y, elist, n, qbuf, s, ok);
    case 3: return launch_apply_p3(op, variant, x, y, elist, n, qbuf, s, ok);
    case 4: return launch_apply_p4(op, variant, x, y, elist, n, qbuf, s, ok);
    case 5: return launch_apply_p5(op, variant, x, y, elist, n, qbuf, s, ok);
    case 6: return launch_apply_p6(op, variant, x, y, elist, n, qbuf, s, ok);
    case 7: return launch_apply_p7(op, variant, x, y, elist, n, qbuf, s, ok);
    case 8: return launch_apply_p8(op, variant, x, y, elist, n, qbuf, s, ok);
    }
    *ok = false;
    return hipSuccess;
}

hipError_t launch_apply_lp_p1(const pa_op *, int, const float *, float *, hipStream_t, bool *);
hipError_t launch_apply_lp_p2(const pa_op *, int, const float *, float *, hipStream_t, bool *);
hipError_t launch_apply_lp_p3(const pa_op *, int, const float *, float *, hipStream_t, bool *);
hipError_t launch_apply_lp_p4(const pa_op *, int, const float *, float *, hipStream_t, bool *);
hipError_t launch_apply_lp_p5(const pa_op *, int, const float *, float *, hipStream_t, bool *);
hipError_t launch_apply_lp_p6(const pa_op *, int, const float *, float *, hipStream_t, bool *);
hipError_t launch_apply_lp_p7(const pa_op *, int, const float *, float *, hipStream_t, bool *);
hipError_t launch_apply_lp_p8(const pa_op *, int, const float *, float *, hipStream_t, bool *);

hipError_t launch_apply_lp(const pa_op *op, int fmt, const float *x, float *y, hipStream_t s, bool *ok)
{
    switch (op->p) {
    case 1: return launch_apply_lp_p1(op, fmt, x, y, s, ok);
    case 2: return launch_apply_lp_p2(op, fmt, x, y, s, ok);
    case 3: return launch_apply_lp_p3(op, fmt, x, y, s, ok);
    case 4: return launch_apply_lp_p4(op, fmt, x, y, s, ok);
    case 5: return launch_apply_lp_p5(op, fmt, x, y, s, ok);
    case 6: return launch_apply_lp_p6(op, fmt, x, y, s, ok);
    case 7: return launch_apply_lp_p7(op, fmt, x, y, s, ok);
    case 8: return launch_apply_lp_p8(op, fmt, x, y, s, ok);
    }
    *ok = false;
    return hipSuccess;
}

bool apply_group_shape_p1(int, int, int, int *, int *);
bool apply_group_shape_p2(int, int, int, int *, int *);
bool apply_group_shape_p3(int, int, int, int *, int *);
bool apply_group_shape_p4(int, int, int, int *, int *);
bool apply_group_shape_p5(int, int, int, int *, int *);
bool apply_group_shape_p6(int, int, int, int *, int *);
bool apply_group_shape_p7(int, int, int, int *, int *);
bool apply_group_shape_p8(int, int, int, int *, int *);

// elements per element group and workgroup size of the kernel that a launch of `variant`
// runs (variant -1: the 16-bit apply), as that kernel's template computes them
static bool apply_group_shape(const pa_op *op, int variant, int *elems, int *threads)
{
    switch (op->p) {
    case 1: return apply_group_shape_p1(op->q, op->ops, variant, elems, threads);
    case 2: return apply_group_shape_p2(op->q, op->ops, variant, elems, threads);
    case 3: return apply_group_shape_p3(op->q, op->ops, variant, elems, threads);
    case 4: return apply_group_shape_p4(op->q, op->ops, variant, elems, threads);
    case 5: return apply_group_shape_p5(op->q, op->ops, variant, elems, threads);
    case 6: return apply_group_shape_p6(op->q, op->ops, variant, elems, threads);
    case 7: return apply_group_shape_p7(op->q, op->ops, variant, elems, threads);
    case 8: return apply_group_shape_p8(op->q, op->ops, variant, elems, threads);
    }
    return false;
}

}  // namespace hexpa

using namespace hexpa;


extern "C" const char *pa_last_error(void) { return g_err.c_str(); }

extern "C" void pa_destroy(pa_op *op)
{
    if (!op) return;
    dfree(op->d_elem_dofs);
    dfree(op->d_qdata);
    dfree(op->d_qdata32);
    dfree(op->d_qbuf);
    dfree(op->d_vert);
    dfree(op->d_hex);
    dfree(op->d_tab);
    dfree(op->d_grid);
    dfree(op->d_ess);
    dfree(op->d_color_elems);
    dfree(op->d_scratch);
    delete op;
}

extern "C" int pa_setup(const pa_mesh_desc *m, int order, int q1d, const pa_coeff_desc *c, uint32_t ops,
                        void *stream, pa_op **out)
{
    PA_TRY
    if (!out) return arg_error("pa_setup: out is NULL");
    *out = nullptr;
    if (!m || !m->vert_xyz || !m->hex || m->nvert <= 0 || m->nelem <= 0)
        return arg_error("pa_setup: mesh descriptor incomplete");
    if (order < 1 || order > kMaxP) {
        set_error("pa_setup: order must be in [1, 8]");
        return PA_ERR_UNSUPPORTED;
    }
    if (q1d != order + 1 && q1d != order + 2) {
        set_error("pa_setup: q1d must be order+1 or order+2");
        return PA_ERR_UNSUPPORTED;
    }
    if (ops < 1 || ops > 3) return arg_error("pa_setup: ops must be PA_MASS, PA_DIFFUSION or both");
    if (c && c->kind == PA_COEFF_GRID && (!c->grid || c->gx < 2 || c->gy < 2 || c->gz < 2))
        return arg_error("pa_setup: grid coefficient needs grid and gx, gy, gz >= 2");
    if (c && (c->kind < PA_COEFF_CONST || c->kind > PA_COEFF_GRID)) return arg_error("pa_setup: unknown coefficient kind");
    hipStream_t s = as_stream(stream);

    std::unique_ptr<pa_op, void (*)(pa_op *)> op(new pa_op, pa_destroy);
    op->p = order; op->d = order + 1; op->q = q1d; op->ops = (int)ops;
    // default contraction unit: the faster one measured on MI355X for this order and operator
    // (vector ALU up to p = 4, and for the mass operator alone up to p = 6; MFMA above)
    op->variant = (order <= 4 || (ops == PA_MASS && order <= 6)) ? PA_VARIANT_VALU : PA_VARIANT_MFMA;
    op->ncomp = (ops & PA_DIFFUSION) ? ((ops & PA_MASS) ? 7 : 6) : 1;
    op->nelem = m->nelem; op->nvert = m->nvert;
    std::string terr;
    if (!make_tables(order, q1d, op->tab, terr)) return arg_error(terr.c_str());

    const int d = op->d, d3 = d * d * d;
    const int64_t nel = m->nelem;
    std::vector<int32_t> ed((size_t)nel * d3);
    std::vector<uint8_t> marker;
    if (m->nx > 0) {
        const int64_t nx = m->nx, ny = m->ny, nz = m->nz;
        if (ny <= 0 || nz <= 0 || nx * ny * nz != nel) return arg_error("pa_setup: nx*ny*nz != nelem");
        const int64_t Mx = nx * order + 1, My = ny * order + 1, Mz = nz * order + 1;
        if (Mx * My * Mz > INT32_MAX) return arg_error("pa_setup: too many DOFs for int32 indices");
        op->nx = (int)nx; op->ny = (int)ny; op->nz = (int)nz;
        op->ndof = (int)(Mx * My * Mz);
        for (int64_t e = 0; e < nel; ++e) {
            const int64_t ex = e % nx, ey = (e / nx) % ny, ez = e / (nx * ny);
            int32_t *dst = &ed[(size_t)e * d3];
            for (int k = 0; k < d; ++k)
                for (int j = 0; j < d; ++j)
                    for (int i = 0; i < d; ++i)
                        dst[i + d * (j + d * k)] =
                            (int32_t)((ex * order + i) + Mx * ((ey * order + j) + My * (ez * order + k)));
        }
        if (m->ess_mode == 1) {
            marker.assign((size_t)op->ndof, 0);
            for (int64_t K = 0; K < Mz; ++K)
                for (int64_t J = 0; J < My; ++J)
                    for (int64_t I = 0; I < Mx; ++I)
                        if (I == 0 || J == 0 || K == 0 || I == Mx - 1 || J == My - 1 || K == Mz - 1)
                            marker[(size_t)(I + Mx * (J + My * K))] = 1;
        }
    } else {
        if (!m->elem_dofs || m->ndof <= 0) return arg_error("pa_setup: unstructured mesh needs elem_dofs and ndof");
        op->ndof = m->ndof;
        std::memcpy(ed.data(), m->elem_dofs, ed.size() * sizeof(int32_t));
        for (int32_t v : ed)
            if (v < 0 || v >= m->ndof) return arg_error("pa_setup: elem_dofs entry out of [0, ndof)");
        if (m->ess_mode == 1) return arg_error("pa_setup: ess_mode 1 needs a structured box");
    }
    if (m->ess_mode == 2) {
        if (!m->ess_marker) return arg_error("pa_setup: ess_mode 2 needs ess_marker");
        marker.assign(m->ess_marker, m->ess_marker + op->ndof);
    } else if (m->ess_mode != 0 && m->ess_mode != 1) {
        return arg_error("pa_setup: unknown ess_mode");
    }
    std::vector<int32_t> ess;
    for (size_t i = 0; i < marker.size(); ++i)
        if (marker[i]) ess.push_back((int32_t)i);
    op->ness = (int)ess.size();
    for (int32_t h : std::vector<int32_t>(m->hex, m->hex + 8 * nel))
        if (h < 0 || h >= m->nvert) return arg_error("pa_setup: hex vertex index out of range");

    // colour classes (structured boxes): colour = parity of (ex, ey, ez)
    std::vector<int32_t> colors;
    if (op->nx > 0) {
        std::vector<std::vector<int32_t>> cl(8);
        for (int64_t e = 0; e < nel; ++e) {
            const int64_t ex = e % op->nx, ey = (e / op->nx) % op->ny, ez = e / ((int64_t)op->nx * op->ny);
            cl[(ex & 1) + 2 * (ey & 1) + 4 * (ez & 1)].push_back((int32_t)e);
        }
        op->color_off[0] = 0;
        for (int k = 0; k < 8; ++k) {
            colors.insert(colors.end(), cl[k].begin(), cl[k].end());
            op->color_off[k + 1] = (int)colors.size();
        }
    }

    DevTables ht;
    std::memset(&ht, 0, sizeof(ht));
    for (int a = 0; a < q1d; ++a) {
        ht.w[a] = op->tab.qwts[a];
        ht.x[a] = op->tab.qpts[a];
        for (int i = 0; i < d; ++i) {
            ht.B[a * d + i] = op->tab.B[(size_t)a * d + i];
            ht.G[a * d + i] = op->tab.G[(size_t)a * d + i];
        }
    }
    for (int i = 0; i < d; ++i) ht.nodes[i] = op->tab.nodes[i];

    const int q3 = q1d * q1d * q1d;
    HIP_OK(hipGetDevice(&op->device));
    HIP_OK(dalloc(&op->d_elem_dofs, ed.size()));
    HIP_OK(dalloc(&op->d_qdata, (size_t)nel * op->ncomp * q3));
    HIP_OK(dalloc(&op->d_vert, (size_t)m->nvert * 3));
    HIP_OK(dalloc(&op->d_hex, (size_t)nel * 8));
    HIP_OK(dalloc(&op->d_tab, 1));
    HIP_OK(dalloc(&op->d_scratch, (size_t)op->ndof));
    op->scratch_len = (size_t)op->ndof;
    HIP_OK(hipMemcpy(op->d_elem_dofs, ed.data(), ed.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(op->d_vert, m->vert_xyz, (size_t)m->nvert * 3 * sizeof(double), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(op->d_hex, m->hex, (size_t)nel * 8 * sizeof(int32_t), hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(op->d_tab, &ht, sizeof(ht), hipMemcpyHostToDevice));
    if (!ess.empty()) {
        HIP_OK(dalloc(&op->d_ess, ess.size()));
        HIP_OK(hipMemcpy(op->d_ess, ess.data(), ess.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    if (!colors.empty()) {
        HIP_OK(dalloc(&op->d_color_elems, colors.size()));
        HIP_OK(hipMemcpy(op->d_color_elems, colors.data(), colors.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    }
    CoeffDev cf{PA_COEFF_CONST, 1.0, 0.0, 0.0, nullptr, 0, 0, 0};
    if (c) {
        cf.kind = c->kind; cf.value = c->value; cf.amp = c->amp; cf.freq = c->freq;
        if (c->kind == PA_COEFF_GRID) {
            const size_t ng = (size_t)c->gx * c->gy * c->gz;
            HIP_OK(dalloc(&op->d_grid, ng));
            HIP_OK(hipMemcpy(op->d_grid, c->grid, ng * sizeof(double), hipMemcpyHostToDevice));
            cf.grid = op->d_grid; cf.gx = c->gx; cf.gy = c->gy; cf.gz = c->gz;
        }
    }
    op->coeff = cf;
    int *d_bad = nullptr;
    HIP_OK(hipMalloc((void **)&d_bad, sizeof(int)));
    HIP_OK(hipMemsetAsync(d_bad, 0, sizeof(int), s));
    HIP_OK(launch_setup_qdata(op.get(), cf, d_bad, s));
    int bad = 0;
    HIP_OK(hipMemcpyAsync(&bad, d_bad, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    dfree(d_bad);
    if (bad) {
        set_error("pa_setup: an element has det J <= 0 at a quadrature point");
        return PA_ERR_MESH;
    }
    *out = op.release();
    return PA_OK;
    PA_CATCH
}

int hexpa::do_apply(pa_op *op, int variant, const double *x, double *y, hipStream_t s, bool zero_first)
{
    bool ok = true;
    if (zero_first) HIP_OK(vec_fill(y, 0.0, op->ndof, s));
    if (variant == PA_VARIANT_MFMA_COLORED) {
        if (!op->d_color_elems) {
            set_error("coloured apply needs a structured box mesh");
            return PA_ERR_UNSUPPORTED;
        }
        for (int c = 0; c < 8 && ok; ++c) {
            const int n = op->color_off[c + 1] - op->color_off[c];
            HIP_OK(launch_apply(op, variant, x, y, op->d_color_elems + op->color_off[c], n, s, &ok));
        }
    } else {
        if ((variant == PA_VARIANT_MFMA_UNFUSED || variant == PA_VARIANT_VALU_UNFUSED) && !op->d_qbuf) {
            const int ng = (op->ops & 2) ? ((op->ops & 1) ? 4 : 3) : 1;
            HIP_OK(dalloc(&op->d_qbuf, (size_t)op->nelem * ng * op->q * op->q * op->q));
        }
        HIP_OK(launch_apply(op, variant, x, y, nullptr, op->nelem, s, &ok));
    }
    if (!ok) {
        set_error("apply kernel not instantiated for this (p, q1d, ops)");
        return PA_ERR_UNSUPPORTED;
    }
    return PA_OK;
}

extern "C" int pa_apply(pa_op *op, const double *x, double *y, void *stream)
{
    PA_TRY
    if (!op || !x || !y) return arg_error("pa_apply: NULL argument");
    if (x == y) return arg_error("pa_apply: x and y must not alias");
    return do_apply(op, op->variant, x, y, as_stream(stream));
    PA_CATCH
}

extern "C" int pa_apply_add(pa_op *op, const double *x, double *y, void *stream)
{
    PA_TRY
    if (!op || !x || !y) return arg_error("pa_apply_add: NULL argument");
    if (x == y) return arg_error("pa_apply_add: x and y must not alias");
    return do_apply(op, op->variant, x, y, as_stream(stream), false);
    PA_CATCH
}

// y = A_c x; uses op->d_scratch for the masked input.
int hexpa::do_apply_constrained(pa_op *op, const double *x, double *y, hipStream_t s)
{
    if (op->ness == 0) return do_apply(op, op->variant, x, y, s);
    HIP_OK(vec_copy(op->d_scratch, x, op->ndof, s));
    HIP_OK(vec_zero_list(op->d_scratch, op->d_ess, op->ness, s));
    int rc = do_apply(op, op->variant, op->d_scratch, y, s);
    if (rc) return rc;
    HIP_OK(vec_copy_list(y, x, op->d_ess, op->ness, s));
    return PA_OK;
}

extern "C" int pa_apply_constrained(pa_op *op, const double *x, double *y, void *stream)
{
    PA_TRY
    if (!op || !x || !y) return arg_error("pa_apply_constrained: NULL argument");
    if (x == y) return arg_error("pa_apply_constrained: x and y must not alias");
    return do_apply_constrained(op, x, y, as_stream(stream));
    PA_CATCH
}

extern "C" int pa_diag(pa_op *op, double *dg, int constrained, void *stream)
{
    PA_TRY
    if (!op || !dg) return arg_error("pa_diag: NULL argument");
    hipStream_t s = as_stream(stream);
    HIP_OK(launch_diag(op, dg, s));
    if (constrained && op->ness) HIP_OK(vec_set_list(dg, 1.0, op->d_ess, op->ness, s));
    return PA_OK;
    PA_CATCH
}

extern "C" int pa_load(pa_op *op, const double *f_qp, double *b, void *stream)
{
    PA_TRY
    if (!op || !f_qp || !b) return arg_error("pa_load: NULL argument");
    HIP_OK(launch_load(op, f_qp, b, as_stream(stream)));
    return PA_OK;
    PA_CATCH
}

extern "C" int pa_qpoints(pa_op *op, double *xyz, void *stream)
{
    PA_TRY
    if (!op || !xyz) return arg_error("pa_qpoints: NULL argument");
    HIP_OK(launch_qpoints(op, xyz, as_stream(stream)));
    return PA_OK;
    PA_CATCH
}

extern "C" int pa_nodes(pa_op *op, double *xyz, void *stream)
{
    PA_TRY
    if (!op || !xyz) return arg_error("pa_nodes: NULL argument");
    HIP_OK(launch_nodes(op, xyz, as_stream(stream)));
    return PA_OK;
    PA_CATCH
}

extern "C" int pa_get_elem_dofs(pa_op *op, int32_t *host_out)
{
    PA_TRY
    if (!op || !host_out) return arg_error("pa_get_elem_dofs: NULL argument");
    HIP_OK(hipMemcpy(host_out, op->d_elem_dofs, (size_t)op->nelem * op->d * op->d * op->d * sizeof(int32_t),
                     hipMemcpyDeviceToHost));
    return PA_OK;
    PA_CATCH
}

extern "C" int pa_get_ess(pa_op *op, int32_t *host_out)
{
    PA_TRY
    if (!op || (!host_out && op->ness)) return arg_error("pa_get_ess: NULL argument");
    if (op->ness) HIP_OK(hipMemcpy(host_out, op->d_ess, (size_t)op->ness * sizeof(int32_t), hipMemcpyDeviceToHost));
    return PA_OK;
    PA_CATCH
}

extern "C" int pa_set_variant(pa_op *op, int variant)
{
    if (!op) return arg_error("pa_set_variant: NULL op");
    if (variant < PA_VARIANT_MFMA || variant > PA_VARIANT_VALU_MF) return arg_error("pa_set_variant: unknown variant");
    if (variant == PA_VARIANT_MFMA_COLORED && !op->d_color_elems) {
        set_error("pa_set_variant: coloured apply needs a structured box mesh");
        return PA_ERR_UNSUPPORTED;
    }
    op->variant = variant;
    return PA_OK;
}

extern "C" int pa_set_grid_cap(pa_op *op, int max_workgroups)
{
    if (!op) return arg_error("pa_set_grid_cap: NULL op");
    if (max_workgroups < 0) return arg_error("pa_set_grid_cap: max_workgroups must be >= 0");
    op->grid_cap = max_workgroups;
    return PA_OK;
}

extern "C" int pa_info(const pa_op *op, pa_info_t *info)
{
    if (!op || !info) return arg_error("pa_info: NULL argument");
    info->p = op->p; info->q1d = op->q; info->ops = op->ops; info->nelem = op->nelem; info->ndof = op->ndof;
    info->ness = op->ness; info->ncomp = op->ncomp; info->variant = op->variant;
    const int d = op->d, q = op->q;
    const int ncomp = op->ncomp;
    int elems = 1, threads = 256;
    if (!apply_group_shape(op, op->variant, &elems, &threads)) return arg_error("pa_info: no kernel for this operator");
    info->elems_per_block = elems;
    info->threads_per_block = threads;
    info->qdata_bytes = (int64_t)op->nelem * ncomp * q * q * q * 8;
    info->map_bytes = (int64_t)op->nelem * d * d * d * 4;
    return PA_OK;
}

extern "C" int pa_debug_mfma_f64(int shape, const double *A, const double *B, double *D, void *stream)
{
    if (!A || !B || !D) return arg_error("pa_debug_mfma_f64: NULL argument");
    if (shape != 4 && shape != 16) return arg_error("pa_debug_mfma_f64: shape must be 4 or 16");
    HIP_OK(launch_debug_mfma(shape, A, B, D, as_stream(stream)));
    return PA_OK;
}

extern "C" int pa_debug_mfma16(int bf16, const float *A, const float *B, float *D, void *stream)
{
    if (!A || !B || !D) return arg_error("pa_debug_mfma16: NULL argument");
    HIP_OK(launch_debug_mfma16(bf16 ? 1 : 0, A, B, D, as_stream(stream)));
    return PA_OK;
}

// ------------------------------------------------------------------ mixed-precision apply
static int ensure_qdata32(pa_op *op, hipStream_t s)
{
    if (op->d_qdata32) return PA_OK;
    const int64_t n = (int64_t)op->nelem * op->ncomp * op->q * op->q * op->q;
    HIP_OK(dalloc(&op->d_qdata32, (size_t)n));
    HIP_OK(vec_to_f32(op->d_qdata32, op->d_qdata, 1.0, n, s));
    return PA_OK;
}

// y = A x with the 16-bit apply; zero_first = false: y already holds zeros (or a sum to add to)
static int do_apply_lp(pa_op *op, const float *x, float *y, int fmt, hipStream_t s, bool zero_first = true)
{
    int rc = ensure_qdata32(op, s);
    if (rc) return rc;
    bool ok = true;
    if (zero_first) HIP_OK(vec_fill(y, 0.0f, op->ndof, s));
    HIP_OK(launch_apply_lp(op, fmt, x, y, s, &ok));
    if (!ok) {
        set_error("mixed-precision apply not instantiated for this (p, q1d, ops)");
        return PA_ERR_UNSUPPORTED;
    }
    return PA_OK;
}

extern "C" int pa_apply_lp(pa_op *op, const float *x, float *y, int fmt, void *stream)
{
    PA_TRY
    if (!op || !x || !y) return arg_error("pa_apply_lp: NULL argument");
    if ((const void *)x == (const void *)y) return arg_error("pa_apply_lp: x and y must not alias");
    if (fmt != PA_LP_FP16 && fmt != PA_LP_BF16) return arg_error("pa_apply_lp: fmt must be PA_LP_FP16 or PA_LP_BF16");
    return do_apply_lp(op, x, y, fmt, as_stream(stream));
    PA_CATCH
}

// ------------------------------------------------------------------ CG
namespace {
// Device buffers of one (P)CG run in vector type T; sums and scalars are FP64.
template <class T>
struct PcgWork {
    T *r = nullptr, *p = nullptr, *Ap = nullptr;
    double *partial = nullptr, *partial2 = nullptr, *hist = nullptr, *tmp = nullptr;
    CgScalars *sc = nullptr;
    double *h_hist = nullptr;  // pinned: 2 slots x (r.r, breakdown)
    hipEvent_t ev[2] = {nullptr, nullptr};
    int max_it = 0;
    hipError_t init(int64_t n, int max_it_)
    {
        max_it = max_it_;
        hipError_t e;
        if ((e = dalloc(&r, n)) || (e = dalloc(&p, n)) || (e = dalloc(&Ap, n)) || (e = dalloc(&partial, 2 * kRedBlocks)) ||
            (e = dalloc(&partial2, 2 * kRedBlocks)) ||
            (e = dalloc(&hist, 2 * ((size_t)max_it + 2))) || (e = dalloc(&tmp, 4)) || (e = dalloc(&sc, 1)))
            return e;
        if ((e = hipHostMalloc((void **)&h_hist, 4 * sizeof(double), hipHostMallocDefault))) return e;
        if ((e = hipEventCreateWithFlags(&ev[0], hipEventDisableTiming))) return e;
        return hipEventCreateWithFlags(&ev[1], hipEventDisableTiming);
    }
    ~PcgWork()
    {
        dfree(r); dfree(p); dfree(Ap); dfree(partial); dfree(partial2); dfree(hist); dfree(tmp); dfree(sc);
        if (h_hist) (void)hipHostFree(h_hist);
        for (auto &e : ev)
            if (e) (void)hipEventDestroy(e);
    }
};

// Runs step(it) for it = 1, 2, ... from an initialised state (hist[0] = r0.r0 read back
// as rr0); each step records hist[2 it] = r.r and hist[2 it + 1] = breakdown flag.  Stops
// when r.r <= tol2, on breakdown, or after max_it.  The host inspects the residual of the
// previous check while the next iteration is already queued, so the device never idles
// waiting for the host.
template <class T, class StepF>
int lagged_iterate(StepF step, double tol2, int max_it, int check, PcgWork<T> &w, hipStream_t s, double rr0,
                   int *iters, double *rr_out)
{
    double rr = rr0;
    int it = 0, status = PA_ERR_NOT_CONVERGED;
    if (rr <= tol2) status = PA_OK;
    int pending = -1, nchecks = 0;
    while (status == PA_ERR_NOT_CONVERGED && it < max_it) {
        ++it;
        int rc = step(it);
        if (rc) return rc;
        if (it % check == 0 || it == max_it) {
            const int slot = (nchecks++) & 1;
            HIP_OK(hipMemcpyAsync(w.h_hist + 2 * slot, w.hist + 2 * (size_t)it, 2 * sizeof(double),
                                  hipMemcpyDeviceToHost, s));
            HIP_OK(hipEventRecord(w.ev[slot], s));
            if (pending >= 0) {
                HIP_OK(hipEventSynchronize(w.ev[pending]));
                if (w.h_hist[2 * pending + 1] != 0.0) status = PA_ERR_BREAKDOWN;
                else if (w.h_hist[2 * pending] <= tol2) status = PA_OK;
                rr = w.h_hist[2 * pending];
            }
            pending = slot;
        }
    }
    HIP_OK(hipStreamSynchronize(s));
    if (pending >= 0) {
        rr = w.h_hist[2 * pending];
        if (w.h_hist[2 * pending + 1] != 0.0) status = PA_ERR_BREAKDOWN;
        else if (rr <= tol2) status = PA_OK;
    }
    *iters = it;
    *rr_out = rr;
    return status;
}

struct NoHook {
    int operator()(int) const { return PA_OK; }
};

// (P)CG iterations (Saad, Alg. 9.1) with Jacobi dinv (nullptr: none) from the state cg_init
// left in w; after(it) runs once iteration it has been enqueued.  apply(p, Ap) must add A p
// into Ap, which holds zeros on entry (the direction update clears it for the next one).
template <class T, class ApplyF, class AfterF = NoHook>
int pcg_iterate(ApplyF apply, T *x, const T *dinv, int64_t n, double tol2, int max_it, int check, PcgWork<T> &w,
                hipStream_t s, double rr0, int *iters, double *rr_out, AfterF after = AfterF())
{
    HIP_OK(vec_fill(w.Ap, T(0), n, s));
    auto step = [&](int it) -> int {
        int rc = apply(w.p, w.Ap);
        if (rc) return rc;
        HIP_OK(cg_pap<T>(w.p, w.Ap, n, w.partial2, s));
        HIP_OK(cg_update_xr<T>(x, w.r, w.p, w.Ap, dinv, n, w.partial2, w.partial, w.sc, s));
        HIP_OK(cg_update_dir<T>(w.p, w.r, dinv, w.Ap, n, w.partial, w.sc, w.hist, it, 1.0, s));
        return after(it);
    };
    return lagged_iterate<T>(step, tol2, max_it, check, w, s, rr0, iters, rr_out);
}
}  // namespace

// y = A p with p vanishing on the essential DOFs (CG invariant): A_c p = A p outside, 0 on
// them.  zero_first = false: y holds zeros on entry (pcg_iterate's contract).
static int cg_apply(pa_op *op, bool constrained, const double *p, double *y, hipStream_t s, bool zero_first = true)
{
    int rc = do_apply(op, op->variant, p, y, s, zero_first);
    if (rc) return rc;
    if (constrained && op->ness) HIP_OK(vec_zero_list(y, op->d_ess, op->ness, s));
    return PA_OK;
}

static int true_residual(pa_op *op, bool con, const double *b, const double *x, double *tmp, double *tmp2,
                         PcgWork<double> &w, double bnorm, hipStream_t s, double *rel)
{
    int rc = con ? do_apply_constrained(op, x, tmp, s) : do_apply(op, op->variant, x, tmp, s);
    if (rc) return rc;
    HIP_OK(cg_init<double>(b, tmp, tmp2, nullptr, op->ndof, w.partial, w.sc, w.hist, s));
    HIP_OK(hipMemcpyAsync(w.h_hist, w.hist, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    *rel = std::sqrt(w.h_hist[0]) / bnorm;
    return PA_OK;
}

static int solve_mixed_ir(pa_op *op, const double *b, double *x, const pa_cg_opts *o, pa_cg_result *res,
                          hipStream_t s, double bnorm, PcgWork<double> &w64, const double *dinv64)
{
    const int64_t n = op->ndof;
    const bool con = o->constrained != 0;
    const int fmt = o->lp_fmt;
    if (fmt != PA_LP_FP16 && fmt != PA_LP_BF16) return arg_error("cg_solve: lp_fmt must be PA_LP_FP16 or PA_LP_BF16");
    const int inner_max = o->inner_max > 0 ? o->inner_max : 200;
    const double inner_rtol = o->inner_rtol > 0.0 ? o->inner_rtol : 1e-2;
    const int check = o->check_every < 1 ? 1 : o->check_every;
    int rc = ensure_qdata32(op, s);
    if (rc) return rc;
    PcgWork<float> w32;
    HIP_OK(w32.init(n, inner_max));
    float *d32 = nullptr, *dinv32 = nullptr;
    HIP_OK(dalloc(&d32, n));
    std::unique_ptr<void, void (*)(void *)> g1(d32, dfree);
    if (dinv64) {
        HIP_OK(dalloc(&dinv32, n));
        HIP_OK(vec_to_f32(dinv32, dinv64, 1.0, n, s));
    }
    std::unique_ptr<void, void (*)(void *)> g2(dinv32, dfree);
    auto apply32 = [&](const float *p, float *y) -> int {
        int r2 = do_apply_lp(op, p, y, fmt, s, false);
        if (r2) return r2;
        if (con && op->ness) HIP_OK(vec_set_list(y, 0.0f, op->d_ess, op->ness, s));
        return PA_OK;
    };
    auto t0 = std::chrono::steady_clock::now();
    int status = PA_ERR_NOT_CONVERGED, outer = 0, inner_total = 0;
    double rel = 0.0;
    for (;;) {
        // FP64 residual r = b - A x and its norm / max-abs scale
        rc = con ? do_apply_constrained(op, x, w64.Ap, s) : do_apply(op, op->variant, x, w64.Ap, s);
        if (rc) return rc;
        HIP_OK(cg_init<double>(b, w64.Ap, w64.r, nullptr, n, w64.partial, w64.sc, w64.hist, s));  // Ap <- b - Ax
        HIP_OK(vec_maxabs(w64.Ap, n, w64.partial, w64.tmp, s));
        HIP_OK(hipMemcpyAsync(w64.h_hist, w64.hist, sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_OK(hipMemcpyAsync(w64.h_hist + 1, w64.tmp, sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        rel = std::sqrt(w64.h_hist[0]) / bnorm;
        const double rmax = w64.h_hist[1];
        if (!std::isfinite(rel)) { status = PA_ERR_BREAKDOWN; break; }
        if (rel <= o->rtol) { status = PA_OK; break; }
        if (outer >= o->max_it) break;
        ++outer;
        // scale the residual by a power of two so its largest entry is in [0.5, 1)
        int ex = 0;
        std::frexp(rmax, &ex);
        const double scale = std::ldexp(1.0, -ex);
        HIP_OK(vec_to_f32(w32.r, w64.Ap, scale, n, s));
        HIP_OK(vec_fill(d32, 0.0f, n, s));
        HIP_OK(cg_init<float>(nullptr, w32.r, w32.p, dinv32, n, w32.partial, w32.sc, w32.hist, s));
        HIP_OK(hipMemcpyAsync(w32.h_hist, w32.hist, sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        const double rr0 = w32.h_hist[0];
        int it_in = 0;
        double rr_in = 0.0;
        int st = pcg_iterate<float>(apply32, d32, dinv32, n, inner_rtol * inner_rtol * rr0, inner_max, check, w32, s,
                                    rr0, &it_in, &rr_in);
        inner_total += it_in;
        if (st == PA_ERR_BREAKDOWN && it_in <= 1) { status = PA_ERR_BREAKDOWN; break; }
        if (st != PA_OK && st != PA_ERR_NOT_CONVERGED && st != PA_ERR_BREAKDOWN) return st;
        HIP_OK(vec_axpy_f32(x, 1.0 / scale, d32, n, s));
    }
    HIP_OK(hipStreamSynchronize(s));
    auto t1 = std::chrono::steady_clock::now();
    res->seconds = std::chrono::duration<double>(t1 - t0).count();
    res->iters = outer;
    res->inner_iters_total = inner_total;
    res->rel_res_recursive = rel;
    double trel = 0.0;
    rc = true_residual(op, con, b, x, w64.Ap, w64.r, w64, bnorm, s, &trel);
    if (rc) return rc;
    res->rel_res_true = trel;
    res->status = status;
    if (status == PA_ERR_NOT_CONVERGED) set_error("cg_solve: max_it refinement steps reached before rtol");
    if (status == PA_ERR_BREAKDOWN) set_error("cg_solve: breakdown in mixed-precision refinement");
    return status;
}

// Flexible CG, FCG(1) (Notay 2000): beta_k = (z_{k+1}, r_{k+1} - r_k) / (z_k, r_k) with a
// variable (here nonlinear) preconditioner z = M(r).  On breakdown it restarts as
// Jacobi-PCG from the current iterate for the remaining iterations.
static int solve_fcg(pa_op *op, const double *b, double *x, const pa_cg_opts *o, pa_cg_result *res, hipStream_t s,
                     double bnorm, PcgWork<double> &w, const double *dinv)
{
    pa_lp *lp = o->lp;
    if (!lp) return arg_error("cg_solve: PA_CG_FCG needs opts->lp");
    if (lp_operator(lp) != op) return arg_error("cg_solve: the pa_lp handle is bound to another operator");
    const int64_t n = op->ndof;
    const bool con = o->constrained != 0;
    const int check = o->check_every < 1 ? 1 : o->check_every;
    double *z = nullptr, *rold = nullptr;
    HIP_OK(dalloc(&z, n));
    std::unique_ptr<void, void (*)(void *)> g1(z, dfree);
    HIP_OK(dalloc(&rold, n));
    std::unique_ptr<void, void (*)(void *)> g2(rold, dfree);
    int rc = con ? do_apply_constrained(op, x, w.r, s) : do_apply(op, op->variant, x, w.r, s);
    if (rc) return rc;
    HIP_OK(cg_init<double>(b, w.r, w.p, nullptr, n, w.partial, w.sc, w.hist, s));  // r = b - A x, hist[0] = r.r
    HIP_OK(hipMemcpyAsync(w.h_hist, w.hist, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    const double rr0 = w.h_hist[0];
    const double tol2 = (o->rtol * bnorm) * (o->rtol * bnorm);
    auto t0 = std::chrono::steady_clock::now();
    rc = lp_precondition(lp, w.r, z, s);
    if (rc) return rc;
    HIP_OK(fcg_direction(z, w.r, nullptr, w.p, n, w.partial, w.sc, s));
    // iterates requested by the caller (training-data capture)
    int cap = 0;
    auto capture = [&](int k) -> int {
        if (cap < o->n_capture && o->capture_at[cap] == k) {
            HIP_OK(vec_copy(o->capture_x + (size_t)cap * n, x, n, s));
            ++cap;
        }
        return PA_OK;
    };
    if ((rc = capture(0))) return rc;
    auto step = [&](int it) -> int {
        int r2 = cg_apply(op, con, w.p, w.Ap, s);
        if (r2) return r2;
        HIP_OK(cg_alpha<double>(w.p, w.Ap, n, w.partial, w.sc, s));
        HIP_OK(fcg_update(x, w.r, rold, w.p, w.Ap, n, w.partial, w.sc, w.hist, it, s));
        if ((r2 = capture(it))) return r2;
        r2 = lp_precondition(lp, w.r, z, s);
        if (r2) return r2;
        HIP_OK(fcg_direction(z, w.r, rold, w.p, n, w.partial, w.sc, s));
        return PA_OK;
    };
    int it = 0;
    double rr = 0.0;
    int status = lagged_iterate<double>(step, tol2, o->max_it, check, w, s, rr0, &it, &rr);
    if (status != PA_OK && status != PA_ERR_NOT_CONVERGED && status != PA_ERR_BREAKDOWN) return status;
    res->fallback = 0;
    if (status == PA_ERR_BREAKDOWN && it < o->max_it) {
        // Jacobi-PCG from the current iterate
        res->fallback = 1;
        rc = con ? do_apply_constrained(op, x, w.r, s) : do_apply(op, op->variant, x, w.r, s);
        if (rc) return rc;
        HIP_OK(cg_init<double>(b, w.r, w.p, dinv, n, w.partial, w.sc, w.hist, s));
        HIP_OK(hipMemcpyAsync(w.h_hist, w.hist, sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        int it2 = 0;
        auto apply64 = [&](const double *p, double *y) { return cg_apply(op, con, p, y, s, false); };
        status = pcg_iterate<double>(apply64, x, dinv, n, tol2, o->max_it - it, check, w, s, w.h_hist[0], &it2, &rr);
        if (status != PA_OK && status != PA_ERR_NOT_CONVERGED && status != PA_ERR_BREAKDOWN) return status;
        it += it2;
    }
    auto t1 = std::chrono::steady_clock::now();
    res->seconds = std::chrono::duration<double>(t1 - t0).count();
    res->iters = it;
    res->rel_res_recursive = std::sqrt(rr) / bnorm;
    double trel = 0.0;
    rc = true_residual(op, con, b, x, w.Ap, w.r, w, bnorm, s, &trel);
    if (rc) return rc;
    res->rel_res_true = trel;
    res->status = status;
    if (status == PA_ERR_NOT_CONVERGED) set_error("cg_solve: max_it reached before rtol");
    if (status == PA_ERR_BREAKDOWN) set_error("cg_solve: breakdown in FCG and in the Jacobi-PCG fallback");
    return status;
}

// One Jacobi-PCG recurrence on FP32 vectors with the 16-bit apply, never restarted;
// every few iterations its residual is replaced by the true FP64 residual ("reliable
// updates", Sleijpen & van der Vorst 1996): x += xh / scale (the FP32 update accumulated
// since the last replacement), r = b - A x in FP64, rh = scale' r with a new power-of-two
// scale, and the direction continues from the old one rescaled by scale' / scale (the
// next beta uses the replaced residual).  Replacement k + 1 comes after a chunk of
// iterations predicted from the convergence rate so far, at most inner_max.
static int solve_mixed_ru(pa_op *op, const double *b, double *x, const pa_cg_opts *o, pa_cg_result *res,
                          hipStream_t s, double bnorm, PcgWork<double> &w64, const double *dinv64)
{
    const int64_t n = op->ndof;
    const bool con = o->constrained != 0;
    const int fmt = o->lp_fmt;
    if (fmt != PA_LP_FP16 && fmt != PA_LP_BF16) return arg_error("cg_solve: lp_fmt must be PA_LP_FP16 or PA_LP_BF16");
    if (!dinv64) return arg_error("cg_solve: MIXED_RU needs the Jacobi diagonal");
    const int kmax = o->inner_max > 0 ? o->inner_max : 100;
    const int max_total = o->max_it;
    int rc = ensure_qdata32(op, s);
    if (rc) return rc;
    PcgWork<float> w32;
    HIP_OK(w32.init(n, max_total + 2));
    float *xh = nullptr, *dinv32 = nullptr;
    HIP_OK(dalloc(&xh, n));
    std::unique_ptr<void, void (*)(void *)> g1(xh, dfree);
    HIP_OK(dalloc(&dinv32, n));
    std::unique_ptr<void, void (*)(void *)> g2(dinv32, dfree);
    HIP_OK(vec_to_f32(dinv32, dinv64, 1.0, n, s));
    CgScalars *hsc = nullptr;
    HIP_OK(hipHostMalloc((void **)&hsc, sizeof(CgScalars), hipHostMallocDefault));
    std::unique_ptr<void, hipError_t (*)(void *)> g3(hsc, hipHostFree);
    // true residual r64 = b - A x (in w64.Ap), its norm and max-abs (host)
    auto true_res = [&](double *rel, double *rmax) -> int {
        int r2 = con ? do_apply_constrained(op, x, w64.Ap, s) : do_apply(op, op->variant, x, w64.Ap, s);
        if (r2) return r2;
        HIP_OK(cg_init<double>(b, w64.Ap, nullptr, nullptr, n, w64.partial, w64.sc, w64.hist, s));
        HIP_OK(vec_maxabs(w64.Ap, n, w64.partial, w64.tmp, s));
        HIP_OK(hipMemcpyAsync(w64.h_hist, w64.hist, sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_OK(hipMemcpyAsync(w64.h_hist + 1, w64.tmp, sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_OK(hipMemcpyAsync(hsc, w32.sc, sizeof(CgScalars), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        *rel = std::sqrt(w64.h_hist[0]) / bnorm;
        *rmax = w64.h_hist[1];
        return PA_OK;
    };
    auto pow2_scale = [](double rmax) {
        int ex = 0;
        std::frexp(rmax, &ex);
        return std::ldexp(1.0, -ex);
    };
    auto t0 = std::chrono::steady_clock::now();
    int status = PA_ERR_NOT_CONVERGED, total = 0, replacements = 0;
    double rel = 0.0, rmax = 0.0;
    static_assert(sizeof(CgScalars) % sizeof(double) == 0, "CgScalars is cleared as doubles");
    HIP_OK(vec_fill(reinterpret_cast<double *>(w32.sc), 0.0, sizeof(CgScalars) / sizeof(double), s));  // rz = 0
    if ((rc = true_res(&rel, &rmax))) return rc;
    if (!std::isfinite(rel)) status = PA_ERR_BREAKDOWN;
    else if (rel <= o->rtol) status = PA_OK;
    double scale = 1.0, rel_prev = rel;
    int chunk_prev = 0, k = kmax;
    bool first = true;
    while (status == PA_ERR_NOT_CONVERGED && total < max_total) {
        // replace the recursive residual: rh = scale' r64, direction rescaled by scale' / scale
        const double ns = pow2_scale(rmax);
        const double f = first ? 1.0 : ns / scale;
        HIP_OK(vec_to_f32(w32.r, w64.Ap, ns, n, s));
        HIP_OK(vec_fill(xh, 0.0f, n, s));
        HIP_OK(cg_rz_partials<float>(w32.r, dinv32, n, w32.partial, s));
        HIP_OK(cg_update_dir<float>(w32.p, w32.r, dinv32, w32.Ap, n, w32.partial, w32.sc, w32.hist, total, f, s));
        scale = ns;
        first = false;
        // chunk length from the observed rate (iterations per factor of reduction)
        if (chunk_prev > 0 && rel < rel_prev && rel_prev > 0.0) {
            const double per_it = std::log(rel / rel_prev) / chunk_prev;  // < 0
            const int need = (int)std::ceil(std::log(o->rtol / rel) / per_it);
            k = std::max(8, std::min(kmax, need + 2));
        }
        k = std::min(k, max_total - total);
        for (int j = 1; j <= k; ++j) {
            rc = do_apply_lp(op, w32.p, w32.Ap, fmt, s, false);
            if (rc) return rc;
            if (con && op->ness) HIP_OK(vec_set_list(w32.Ap, 0.0f, op->d_ess, op->ness, s));
            HIP_OK(cg_pap<float>(w32.p, w32.Ap, n, w32.partial2, s));
            HIP_OK(cg_update_xr<float>(xh, w32.r, w32.p, w32.Ap, dinv32, n, w32.partial2, w32.partial, w32.sc, s));
            if (j < k)
                HIP_OK(cg_update_dir<float>(w32.p, w32.r, dinv32, w32.Ap, n, w32.partial, w32.sc, w32.hist, total + j,
                                            1.0, s));
        }
        total += k;
        HIP_OK(vec_axpy_f32(x, 1.0 / scale, xh, n, s));
        rel_prev = rel;
        chunk_prev = k;
        ++replacements;
        if ((rc = true_res(&rel, &rmax))) return rc;
        if (!std::isfinite(rel) || hsc->breakdown) { status = PA_ERR_BREAKDOWN; break; }
        if (rel <= o->rtol) status = PA_OK;
    }
    auto t1 = std::chrono::steady_clock::now();
    res->seconds = std::chrono::duration<double>(t1 - t0).count();
    res->iters = replacements;
    res->inner_iters_total = total;
    res->rel_res_recursive = rel;
    double trel = 0.0;
    rc = true_residual(op, con, b, x, w64.Ap, w64.r, w64, bnorm, s, &trel);
    if (rc) return rc;
    res->rel_res_true = trel;
    res->status = status;
    if (status == PA_ERR_NOT_CONVERGED) set_error("cg_solve: max_it iterations reached before rtol");
    if (status == PA_ERR_BREAKDOWN) set_error("cg_solve: breakdown in the reliable-update mixed-precision CG");
    return status;
}

// FP64 FCG(1) whose preconditioner is the inner mixed-precision solve: z = M(r) with
// M(r) = d / scale, d ~ A^{-1}(scale r) from Jacobi-PCG on FP32 vectors with the 16-bit
// apply (scale = power of two putting max |r| in [0.5, 1)).
static int solve_mixed_fcg(pa_op *op, const double *b, double *x, const pa_cg_opts *o, pa_cg_result *res,
                           hipStream_t s, double bnorm, PcgWork<double> &w, const double *dinv64)
{
    const int64_t n = op->ndof;
    const bool con = o->constrained != 0;
    const int fmt = o->lp_fmt;
    if (fmt != PA_LP_FP16 && fmt != PA_LP_BF16) return arg_error("cg_solve: lp_fmt must be PA_LP_FP16 or PA_LP_BF16");
    const int inner_max = o->inner_max > 0 ? o->inner_max : 200;
    const double inner_rtol = o->inner_rtol > 0.0 ? o->inner_rtol : 1e-2;
    const int check = o->check_every < 1 ? 1 : o->check_every;
    int rc = ensure_qdata32(op, s);
    if (rc) return rc;
    PcgWork<float> w32;
    HIP_OK(w32.init(n, inner_max));
    float *d32 = nullptr, *dinv32 = nullptr;
    double *z = nullptr, *rold = nullptr, *tmp = nullptr;
    HIP_OK(dalloc(&d32, n));
    std::unique_ptr<void, void (*)(void *)> g1(d32, dfree);
    HIP_OK(dalloc(&dinv32, n));
    std::unique_ptr<void, void (*)(void *)> g2(dinv32, dfree);
    HIP_OK(dalloc(&z, n));
    std::unique_ptr<void, void (*)(void *)> g3(z, dfree);
    HIP_OK(dalloc(&rold, n));
    std::unique_ptr<void, void (*)(void *)> g4(rold, dfree);
    HIP_OK(dalloc(&tmp, 2));
    std::unique_ptr<void, void (*)(void *)> g5(tmp, dfree);
    HIP_OK(vec_to_f32(dinv32, dinv64, 1.0, n, s));
    auto apply32 = [&](const float *p, float *y) -> int {
        int r2 = do_apply_lp(op, p, y, fmt, s, false);
        if (r2) return r2;
        if (con && op->ness) HIP_OK(vec_set_list(y, 0.0f, op->d_ess, op->ness, s));
        return PA_OK;
    };
    int inner_total = 0;
    double *hbuf = w32.h_hist;  // pinned scratch for the scale read-back (slots 2, 3 are free here)
    auto precondition = [&](const double *r, double *zout) -> int {
        HIP_OK(vec_maxabs(r, n, w.partial, tmp, s));
        HIP_OK(hipMemcpyAsync(hbuf + 2, tmp, sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        const double rmax = hbuf[2];
        HIP_OK(vec_fill(zout, 0.0, n, s));
        if (!(rmax > 0.0) || !std::isfinite(rmax)) return PA_OK;
        int ex = 0;
        std::frexp(rmax, &ex);
        const double scale = std::ldexp(1.0, -ex);
        HIP_OK(vec_to_f32(w32.r, r, scale, n, s));
        HIP_OK(vec_fill(d32, 0.0f, n, s));
        HIP_OK(cg_init<float>(nullptr, w32.r, w32.p, dinv32, n, w32.partial, w32.sc, w32.hist, s));
        HIP_OK(hipMemcpyAsync(hbuf, w32.hist, sizeof(double), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        const double rr0 = hbuf[0];
        int it_in = 0;
        double rr_in = 0.0;
        int st = pcg_iterate<float>(apply32, d32, dinv32, n, inner_rtol * inner_rtol * rr0, inner_max, check, w32, s,
                                    rr0, &it_in, &rr_in);
        inner_total += it_in;
        if (st != PA_OK && st != PA_ERR_NOT_CONVERGED && st != PA_ERR_BREAKDOWN) return st;
        HIP_OK(vec_axpy_f32(zout, 1.0 / scale, d32, n, s));
        return PA_OK;
    };
    // r = b - A x; z = M(r); p = z
    rc = con ? do_apply_constrained(op, x, w.r, s) : do_apply(op, op->variant, x, w.r, s);
    if (rc) return rc;
    HIP_OK(cg_init<double>(b, w.r, w.p, nullptr, n, w.partial, w.sc, w.hist, s));
    HIP_OK(hipMemcpyAsync(w.h_hist, w.hist, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    const double rr0 = w.h_hist[0];
    const double tol2 = (o->rtol * bnorm) * (o->rtol * bnorm);
    auto t0 = std::chrono::steady_clock::now();
    int it = 0, status = PA_OK;
    double rr = rr0;
    if (rr0 > tol2) {
        rc = precondition(w.r, z);
        if (rc) return rc;
        HIP_OK(fcg_direction(z, w.r, nullptr, w.p, n, w.partial, w.sc, s));
        // outer iterations, each checked at once: the inner solve synchronises with the host anyway
        status = PA_ERR_NOT_CONVERGED;
        while (it < o->max_it) {
            ++it;
            rc = cg_apply(op, con, w.p, w.Ap, s);
            if (rc) return rc;
            HIP_OK(cg_alpha<double>(w.p, w.Ap, n, w.partial, w.sc, s));
            HIP_OK(fcg_update(x, w.r, rold, w.p, w.Ap, n, w.partial, w.sc, w.hist, it, s));
            HIP_OK(hipMemcpyAsync(w.h_hist, w.hist + 2 * (size_t)it, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
            HIP_OK(hipStreamSynchronize(s));
            rr = w.h_hist[0];
            if (w.h_hist[1] != 0.0) { status = PA_ERR_BREAKDOWN; break; }
            if (rr <= tol2) { status = PA_OK; break; }
            rc = precondition(w.r, z);
            if (rc) return rc;
            HIP_OK(fcg_direction(z, w.r, rold, w.p, n, w.partial, w.sc, s));
        }
    }
    HIP_OK(hipStreamSynchronize(s));
    auto t1 = std::chrono::steady_clock::now();
    res->seconds = std::chrono::duration<double>(t1 - t0).count();
    res->iters = it;
    res->inner_iters_total = inner_total;
    res->rel_res_recursive = std::sqrt(rr) / bnorm;
    double trel = 0.0;
    rc = true_residual(op, con, b, x, w.Ap, w.r, w, bnorm, s, &trel);
    if (rc) return rc;
    res->rel_res_true = trel;
    res->status = status;
    if (status == PA_ERR_NOT_CONVERGED) set_error("cg_solve: max_it outer iterations reached before rtol");
    if (status == PA_ERR_BREAKDOWN) set_error("cg_solve: breakdown in the mixed-precision FCG");
    return status;
}

extern "C" int cg_solve(pa_op *op, const double *b, double *x, const pa_cg_opts *o, pa_cg_result *res, void *stream)
{
    PA_TRY
    if (!op || !b || !x || !o || !res) return arg_error("cg_solve: NULL argument");
    if (!(o->rtol > 0.0) || o->max_it < 1) return arg_error("cg_solve: need rtol > 0 and max_it >= 1");
    if (o->mode != PA_CG_PLAIN && o->mode != PA_CG_JACOBI && o->mode != PA_CG_MIXED_IR && o->mode != PA_CG_FCG &&
        o->mode != PA_CG_MIXED_FCG && o->mode != PA_CG_MIXED_RU)
        return arg_error("cg_solve: unknown mode");
    if (o->mode == PA_CG_FCG && !o->lp) return arg_error("cg_solve: PA_CG_FCG needs opts->lp");
    if (o->mode == PA_CG_FCG && lp_operator(o->lp) != op)
        return arg_error("cg_solve: the pa_lp handle is bound to another operator");
    if (o->n_capture < 0 ||
        (o->n_capture > 0 && ((o->mode != PA_CG_JACOBI && o->mode != PA_CG_FCG) || !o->capture_at || !o->capture_x)))
        return arg_error("cg_solve: capture needs PA_CG_JACOBI or PA_CG_FCG, capture_at and capture_x");
    for (int j = 0; j < o->n_capture; ++j)
        if (o->capture_at[j] < 0 || (j > 0 && o->capture_at[j] <= o->capture_at[j - 1]))
            return arg_error("cg_solve: capture_at must be ascending and >= 0");
    std::memset(res, 0, sizeof(*res));
    hipStream_t s = as_stream(stream);
    const int64_t n = op->ndof;
    const bool con = o->constrained != 0;
    const int check = o->check_every < 1 ? 1 : o->check_every;
    PcgWork<double> w;
    HIP_OK(w.init(n, o->mode == PA_CG_MIXED_IR ? 4 : o->max_it));
    if (o->mode == PA_CG_MIXED_FCG && !(o->max_it >= 1)) return arg_error("cg_solve: max_it must be >= 1");
    double *dinv = nullptr;
    std::unique_ptr<void, void (*)(void *)> gd(nullptr, dfree);
    if (o->mode != PA_CG_PLAIN) {  // Jacobi (also the inner preconditioner of MIXED_IR)
        HIP_OK(dalloc(&dinv, n));
        gd.reset(dinv);
        int rc = pa_diag(op, dinv, con ? 1 : 0, s);
        if (rc) return rc;
        HIP_OK(vec_recip(dinv, dinv, n, s));
    }
    if (con && op->ness) HIP_OK(vec_copy_list(x, b, op->d_ess, op->ness, s));
    HIP_OK(vec_dot<double>(b, b, n, w.partial, w.tmp, s));
    double bb = 0.0;
    HIP_OK(hipMemcpyAsync(&bb, w.tmp, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    const double bnorm = std::sqrt(bb);
    if (bnorm == 0.0) {
        HIP_OK(vec_fill(x, 0.0, n, s));
        HIP_OK(hipStreamSynchronize(s));
        res->status = PA_OK;
        return PA_OK;
    }
    if (o->mode == PA_CG_MIXED_IR) return solve_mixed_ir(op, b, x, o, res, s, bnorm, w, dinv);
    if (o->mode == PA_CG_FCG) return solve_fcg(op, b, x, o, res, s, bnorm, w, dinv);
    if (o->mode == PA_CG_MIXED_FCG) return solve_mixed_fcg(op, b, x, o, res, s, bnorm, w, dinv);
    if (o->mode == PA_CG_MIXED_RU) return solve_mixed_ru(op, b, x, o, res, s, bnorm, w, dinv);

    // r = b - A x, p = M^{-1} r
    int rc = con ? do_apply_constrained(op, x, w.r, s) : do_apply(op, op->variant, x, w.r, s);
    if (rc) return rc;
    HIP_OK(cg_init<double>(b, w.r, w.p, dinv, n, w.partial, w.sc, w.hist, s));
    HIP_OK(hipMemcpyAsync(w.h_hist, w.hist, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    const double tol2 = (o->rtol * bnorm) * (o->rtol * bnorm);
    auto t0 = std::chrono::steady_clock::now();
    int it = 0;
    double rr = 0.0;
    auto apply64 = [&](const double *p, double *y) { return cg_apply(op, con, p, y, s, false); };
    // iterates requested by the caller (training-data capture)
    int cap = 0;
    auto capture = [&](int k) -> int {
        if (cap < o->n_capture && o->capture_at[cap] == k) {
            HIP_OK(vec_copy(o->capture_x + (size_t)cap * n, x, n, s));
            ++cap;
        }
        return PA_OK;
    };
    if ((rc = capture(0))) return rc;
    const int status =
        pcg_iterate<double>(apply64, x, dinv, n, tol2, o->max_it, check, w, s, w.h_hist[0], &it, &rr, capture);
    if (status != PA_OK && status != PA_ERR_NOT_CONVERGED && status != PA_ERR_BREAKDOWN) return status;
    auto t1 = std::chrono::steady_clock::now();
    res->seconds = std::chrono::duration<double>(t1 - t0).count();
    res->iters = it;
    res->rel_res_recursive = std::sqrt(rr) / bnorm;
    double trel = 0.0;
    rc = true_residual(op, con, b, x, w.Ap, w.r, w, bnorm, s, &trel);
    if (rc) return rc;
    res->rel_res_true = trel;
    res->status = status;
    if (status == PA_ERR_NOT_CONVERGED) set_error("cg_solve: max_it reached before rtol");
    if (status == PA_ERR_BREAKDOWN) set_error("cg_solve: breakdown (p^T A p <= 0 or non-finite scalar)");
    return status;
    PA_CATCH
}
