"""Thin ctypes binding of libhhg (include/hhg.h).

Argument marshalling only: every function forwards to the C entry point of
the same name.  Device buffers are passed as torch CUDA tensors (or raw
integer addresses); a non-zero status raises HHGError with the library's
message.  Loading fails loudly when libhhg.so has not been built.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhhg.so")

HHG_OK, HHG_ERR_ARG, HHG_ERR_PREC, HHG_ERR_HIP, HHG_ERR_OOM, HHG_ERR_NOT_CONVERGED, HHG_ERR_STATE = range(7)
HHG_P1P1, HHG_P2P1 = 0, 1
HHG_F64, HHG_F32, HHG_BF16 = 0, 1, 2
HHG_OP_FULL, HHG_OP_A, HHG_OP_BT, HHG_OP_B, HHG_OP_C, HHG_OP_MASS = range(6)
HHG_GS_FWD, HHG_GS_SYM = 0, 1
HHG_SCHUR_SD, HHG_SCHUR_ML = 0, 1

SYMBOLS = [
    "hhg_ctx_create", "hhg_ctx_set_stream", "hhg_ctx_destroy", "hhg_last_error",
    "hhg_mesh_cube", "hhg_mesh_create", "hhg_mesh_info", "hhg_mesh_destroy", "hhg_mesh_set_outflow",
    "hhg_mesh_set_outflow_faces",
    "hhg_hier_create", "hhg_hier_destroy", "hhg_vec_layout", "hhg_vec_from_lattice", "hhg_vec_to_lattice",
    "hhg_apply", "hhg_residual", "hhg_rhs", "hhg_smooth", "hhg_restrict", "hhg_prolong_add",
    "hhg_coarse_solve", "hhg_project_mean_zero", "hhg_copy_boundary", "hhg_estimate_omega", "hhg_norms",
    "hhg_vcycle", "hhg_fmg_solve", "hhg_query_stencil", "hhg_query_interpolation", "hhg_query_umesh", "hhg_dots",
    "hhg_timer_start", "hhg_timer_read", "hhg_dc_solve", "hhg_set_viscosity",
    "hhg_mlp_create", "hhg_mlp_destroy", "hhg_mlp_num_params", "hhg_mlp_set_params", "hhg_mlp_get_params",
    "hhg_mlp_forward", "hhg_mlp_loss_grad", "hhg_mlp_train", "hhg_mlp_train_noalloc", "hhg_mlp_dims", "hhg_coarse_pair", "hhg_hier_set_mlp",
    "hhg_record_pairs", "hhg_recorded_pairs", "hhg_hier_set_fused_sites", "hhg_hier_set_bf16_levels",
]
KF_APPLY, KF_PROW_BND, KF_GS_VERTEX, KF_GS_EDGE, KF_PSTEP, KF_RESTRICT, KF_PROLONG, KF_COARSE, KF_REDUCE, KF_OTHER, \
    KF_MLP, KF_SMALL, KF_NEUMANN, KF_IFACE = range(14)


class HHGError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"libhhg status {status}: {msg}")
        self.status = status


class SolverParams(ctypes.Structure):
    _fields_ = [("nu_pre", ctypes.c_int), ("nu_post", ctypes.c_int), ("nu_inc", ctypes.c_int),
                ("kappa", ctypes.c_int), ("gs", ctypes.c_int), ("xi", ctypes.c_int),
                ("omega_inv", ctypes.c_double), ("extra_cycles", ctypes.c_int), ("rtol", ctypes.c_double),
                ("max_cycles", ctypes.c_int), ("coarse_smooth", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int), ("res_u", ctypes.c_double), ("res_p", ctypes.c_double),
                ("rel_res", ctypes.c_double), ("work_units", ctypes.c_double), ("seconds", ctypes.c_double),
                ("fallbacks", ctypes.c_int)]


_lib = None


def load():
    """Load libhhg.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not built: run __graft_entry__.build() first")
    # The library must share the HIP runtime that torch brings (its device
    # memory and streams are what the library is handed): load torch first, so
    # that the runtime is already in the process when libhhg's dependency is
    # resolved, whichever of the two a caller touches first.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P, I, D, S = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    sig = {
        "hhg_ctx_create": [I, P, P],
        "hhg_ctx_set_stream": [P, P],
        "hhg_ctx_destroy": [P],
        "hhg_mesh_cube": [P, I, P],
        "hhg_mesh_create": [P, P, I, P, I, P],
        "hhg_mesh_info": [P, P, P, P],
        "hhg_mesh_destroy": [P],
        "hhg_mesh_set_outflow": [P, ctypes.c_uint],
        "hhg_mesh_set_outflow_faces": [P, P, I],
        "hhg_hier_create": [P, I, I, I, I, P],
        "hhg_hier_destroy": [P],
        "hhg_vec_layout": [P, I, P, P, P, P],
        "hhg_vec_from_lattice": [P, I, P, P, I],
        "hhg_vec_to_lattice": [P, I, P, P, I],
        "hhg_apply": [P, I, I, P, P, I],
        "hhg_residual": [P, I, P, P, P, I],
        "hhg_rhs": [P, I, P, P, I],
        "hhg_smooth": [P, I, P, P, I, I, I, D, I],
        "hhg_restrict": [P, I, P, P, I],
        "hhg_prolong_add": [P, I, P, P, I],
        "hhg_coarse_solve": [P, P, P, I],
        "hhg_project_mean_zero": [P, I, P, I],
        "hhg_copy_boundary": [P, I, P, P, I],
        "hhg_estimate_omega": [P, I, P, I, P],
        "hhg_norms": [P, I, P, P, P, I],
        "hhg_vcycle": [P, I, P, P, P, I],
        "hhg_fmg_solve": [P, P, P, P, P],
        "hhg_query_stencil": [I, ctypes.c_char, I, I, I, I, I, I, P, P, P],
        "hhg_query_interpolation": [I, I, I, I, I, P, P, P],
        "hhg_query_umesh": [P, I, P, I, ctypes.c_uint, I, I, I, P, P, P, P, P, P, P],
        "hhg_dots": [P, I, P, P, P, P, I],
        "hhg_timer_start": [ctypes.c_uint],
        "hhg_timer_read": [I, P, P, P],
        "hhg_dc_solve": [P, P, P, P, I, I, D, I, P],
        "hhg_set_viscosity": [P, I, P],
        "hhg_mlp_create": [P, I, I, I, I, P],
        "hhg_mlp_destroy": [P],
        "hhg_mlp_num_params": [P, P],
        "hhg_mlp_set_params": [P, P],
        "hhg_mlp_get_params": [P, P],
        "hhg_mlp_forward": [P, P, I, P],
        "hhg_mlp_loss_grad": [P, P, P, I, P, P],
        "hhg_mlp_train": [P, P, P, I, I, I, ctypes.c_float, P, P],
        "hhg_mlp_train_noalloc": [P, P, P, I, I, I, ctypes.c_float, P, P],
        "hhg_mlp_dims": [P, P, P],
        "hhg_coarse_pair": [P, P, P, P],
        "hhg_hier_set_mlp": [P, P, D, D],
        "hhg_record_pairs": [P, P, P, I],
        "hhg_recorded_pairs": [P, P],
        "hhg_hier_set_fused_sites": [P, ctypes.c_long],
        "hhg_hier_set_bf16_levels": [P, I],
    }
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = I
    lib.hhg_last_error.argtypes = []
    lib.hhg_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if isinstance(x, ctypes.c_void_p):
        return x.value
    return ctypes.cast(x, ctypes.c_void_p).value


def _check(st):
    if st != HHG_OK:
        raise HHGError(st, load().hhg_last_error().decode())


def hhg_last_error():
    return load().hhg_last_error().decode()


def hhg_ctx_create(device=0, stream=None):
    out = ctypes.c_void_p()
    _check(load().hhg_ctx_create(device, _ptr(stream), ctypes.byref(out)))
    return out


def hhg_ctx_set_stream(ctx, stream):
    _check(load().hhg_ctx_set_stream(ctx, _ptr(stream)))


def hhg_ctx_destroy(ctx):
    _check(load().hhg_ctx_destroy(ctx))


def hhg_mesh_cube(ctx, macro_refine=0):
    out = ctypes.c_void_p()
    _check(load().hhg_mesh_cube(ctx, macro_refine, ctypes.byref(out)))
    return out


def hhg_mesh_create(ctx, xyz, tet):
    """xyz: (nv, 3) host array of vertex coordinates; tet: (nt, 4) vertex indices."""
    import numpy as np
    x = np.ascontiguousarray(xyz, dtype=np.float64)
    t = np.ascontiguousarray(tet, dtype=np.int32)
    out = ctypes.c_void_p()
    _check(load().hhg_mesh_create(ctx, x.ctypes.data, x.shape[0], t.ctypes.data, t.shape[0], ctypes.byref(out)))
    return out


def hhg_mesh_info(mesh):
    nv, nt, mr = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(load().hhg_mesh_info(mesh, ctypes.byref(nv), ctypes.byref(nt), ctypes.byref(mr)))
    return nv.value, nt.value, mr.value


def hhg_mesh_set_outflow(mesh, faces):
    _check(load().hhg_mesh_set_outflow(mesh, int(faces)))


def hhg_mesh_set_outflow_faces(mesh, tri):
    """tri: (ntri, 3) vertex indices of boundary triangles (unstructured meshes)."""
    import numpy as np
    t = np.ascontiguousarray(np.asarray(tri, dtype=np.int32).reshape(-1, 3))
    _check(load().hhg_mesh_set_outflow_faces(mesh, t.ctypes.data if t.size else None, t.shape[0]))


def hhg_mesh_destroy(mesh):
    _check(load().hhg_mesh_destroy(mesh))


def hhg_hier_create(mesh, disc, lmin, lmax, schur=HHG_SCHUR_SD):
    out = ctypes.c_void_p()
    _check(load().hhg_hier_create(mesh, disc, lmin, lmax, schur, ctypes.byref(out)))
    return out


def hhg_hier_destroy(h):
    _check(load().hhg_hier_destroy(h))


def hhg_vec_layout(h, level):
    N = ctypes.c_int()
    nn, vw, lw = ctypes.c_size_t(), ctypes.c_size_t(), ctypes.c_size_t()
    _check(load().hhg_vec_layout(h, level, ctypes.byref(N), ctypes.byref(nn), ctypes.byref(vw), ctypes.byref(lw)))
    return N.value, nn.value, vw.value, lw.value


def hhg_vec_from_lattice(h, level, src, dst, prec=HHG_F64):
    _check(load().hhg_vec_from_lattice(h, level, _ptr(src), _ptr(dst), prec))


def hhg_vec_to_lattice(h, level, src, dst, prec=HHG_F64):
    _check(load().hhg_vec_to_lattice(h, level, _ptr(src), _ptr(dst), prec))


def hhg_apply(h, level, op, x, y, prec=HHG_F64):
    _check(load().hhg_apply(h, level, op, _ptr(x), _ptr(y), prec))


def hhg_residual(h, level, x, b, r, prec=HHG_F64):
    _check(load().hhg_residual(h, level, _ptr(x), _ptr(b), _ptr(r), prec))


def hhg_rhs(h, level, f, b, prec=HHG_F64):
    _check(load().hhg_rhs(h, level, _ptr(f), _ptr(b), prec))


def hhg_smooth(h, level, x, b, iters, gs, xi, omega_inv, prec=HHG_F64):
    _check(load().hhg_smooth(h, level, _ptr(x), _ptr(b), iters, gs, xi, float(omega_inv), prec))


def hhg_restrict(h, fine_level, rf, rc, prec=HHG_F64):
    _check(load().hhg_restrict(h, fine_level, _ptr(rf), _ptr(rc), prec))


def hhg_prolong_add(h, coarse_level, xc, xf, prec=HHG_F64):
    _check(load().hhg_prolong_add(h, coarse_level, _ptr(xc), _ptr(xf), prec))


def hhg_coarse_solve(h, x, b, prec=HHG_F64):
    _check(load().hhg_coarse_solve(h, _ptr(x), _ptr(b), prec))


def hhg_project_mean_zero(h, level, x, prec=HHG_F64):
    _check(load().hhg_project_mean_zero(h, level, _ptr(x), prec))


def hhg_copy_boundary(h, level, src, dst, prec=HHG_F64):
    _check(load().hhg_copy_boundary(h, level, _ptr(src), _ptr(dst), prec))


def hhg_estimate_omega(h, level, v0, iters=100):
    out = ctypes.c_double()
    _check(load().hhg_estimate_omega(h, level, _ptr(v0), iters, ctypes.byref(out)))
    return out.value


def hhg_norms(h, level, x, prec=HHG_F64):
    nu, np_ = ctypes.c_double(), ctypes.c_double()
    _check(load().hhg_norms(h, level, _ptr(x), ctypes.byref(nu), ctypes.byref(np_), prec))
    return nu.value, np_.value


def hhg_set_viscosity(h, level, nu):
    _check(load().hhg_set_viscosity(h, level, _ptr(nu)))


def hhg_dc_solve(h, x, b, prm, inner_prec=HHG_F32, inner_cycles=1, rtol=1e-12, max_outer=100, check=True):
    """Returns the stats; with check=False a tolerance miss (HHG_ERR_NOT_CONVERGED)
    is reported in the stats instead of raised."""
    st = Stats()
    rc = load().hhg_dc_solve(h, _ptr(x), _ptr(b), ctypes.byref(prm), inner_prec, inner_cycles, float(rtol),
                             max_outer, ctypes.byref(st))
    if rc != HHG_OK and (check or rc != HHG_ERR_NOT_CONVERGED):
        _check(rc)
    return st


def hhg_dots(h, level, x, y, prec=HHG_F64):
    du, dp = ctypes.c_double(), ctypes.c_double()
    _check(load().hhg_dots(h, level, _ptr(x), _ptr(y), ctypes.byref(du), ctypes.byref(dp), prec))
    return du.value, dp.value


def hhg_timer_start(family_mask):
    _check(load().hhg_timer_start(family_mask))


def hhg_timer_read(family):
    ms, n, u = ctypes.c_double(), ctypes.c_int(), ctypes.c_double()
    _check(load().hhg_timer_read(family, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(u)))
    return ms.value, n.value, u.value


def solver_params(nu_pre, nu_post, nu_inc, kappa, gs, xi, omega_inv, extra_cycles=0, rtol=0.0, max_cycles=100,
                  coarse_smooth=0):
    return SolverParams(nu_pre, nu_post, nu_inc, kappa, gs, xi, float(omega_inv), extra_cycles, float(rtol),
                        max_cycles, coarse_smooth)


def hhg_vcycle(h, level, x, b, prm, prec=HHG_F64):
    _check(load().hhg_vcycle(h, level, _ptr(x), _ptr(b), ctypes.byref(prm), prec))


def hhg_fmg_solve(h, x, b_levels, prm, want_stats=True, check=True):
    """Returns the stats; with check=False a tolerance miss (HHG_ERR_NOT_CONVERGED)
    returns them too instead of raising."""
    arr = (ctypes.c_void_p * len(b_levels))(*[_ptr(b) for b in b_levels])
    st = Stats()
    rc = load().hhg_fmg_solve(h, _ptr(x), arr, ctypes.byref(prm), ctypes.byref(st) if want_stats else None)
    if rc != HHG_OK and (check or rc != HHG_ERR_NOT_CONVERGED):
        _check(rc)
    return st


def hhg_query_stencil(disc, kind, group, i, j, k, nbox, max_entries=256):
    """Host-only: the library's row stencil at h = 1 as (codes (n, 4), weights (n, 3))."""
    import numpy as np
    n = ctypes.c_int()
    code = (ctypes.c_int * (4 * max_entries))()
    w = (ctypes.c_double * (3 * max_entries))()
    _check(load().hhg_query_stencil(disc, kind.encode() if isinstance(kind, str) else kind, group, i, j, k, nbox,
                                    max_entries, ctypes.byref(n), code, w))
    m = n.value
    return np.array(code[:4 * m]).reshape(m, 4), np.array(w[:3 * m]).reshape(m, 3)


def hhg_query_interpolation(order, tx, ty, tz, q):
    """Host-only: interpolation weights at (tx, ty, tz)/q in a coarse cube."""
    import numpy as np
    n = ctypes.c_int()
    code = (ctypes.c_int * 40)()
    w = (ctypes.c_double * 10)()
    _check(load().hhg_query_interpolation(order, tx, ty, tz, q, ctypes.byref(n), code, w))
    m = n.value
    return np.array(code[:4 * m]).reshape(m, 4), np.array(w[:m])


def hhg_query_umesh(xyz, tet, level, schur=HHG_SCHUR_SD, max_unknowns=0, outflow=0):
    """Host-only: tables of one level of an unstructured mesh.  Returns a dict
    with nnodes, ncolours, nunk, pos (nnodes, 3), colour (nnodes,),
    schur_diag (nnodes,) and K (nunk, nunk) or None."""
    import numpy as np
    x = np.ascontiguousarray(xyz, dtype=np.float64)
    t = np.ascontiguousarray(tet, dtype=np.int32)
    nn, nc, nu = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    lib = load()
    args = (x.ctypes.data, x.shape[0], t.ctypes.data, t.shape[0], int(outflow), level, schur)
    _check(lib.hhg_query_umesh(*args, 0, ctypes.byref(nn), ctypes.byref(nc), ctypes.byref(nu),
                               None, None, None, None))
    n = nn.value
    pos = np.zeros((n, 3))
    col = np.zeros(n, dtype=np.int32)
    sd = np.zeros(n)
    K = np.zeros((nu.value, nu.value)) if 0 < nu.value <= max_unknowns else None
    _check(lib.hhg_query_umesh(*args, max_unknowns, ctypes.byref(nn), ctypes.byref(nc), ctypes.byref(nu),
                               pos.ctypes.data, col.ctypes.data, sd.ctypes.data,
                               None if K is None else K.ctypes.data))
    return {"nnodes": n, "ncolours": nc.value, "nunk": nu.value, "pos": pos, "colour": col, "schur_diag": sd,
            "K": K}


# ------------------------------------------------------------ learned coarse solve
def hhg_mlp_create(ctx, n_in, n_hidden, n_out, max_batch):
    out = ctypes.c_void_p()
    _check(load().hhg_mlp_create(ctx, n_in, n_hidden, n_out, max_batch, ctypes.byref(out)))
    return out


def hhg_mlp_destroy(m):
    _check(load().hhg_mlp_destroy(m))


def hhg_mlp_num_params(m):
    n = ctypes.c_size_t()
    _check(load().hhg_mlp_num_params(m, ctypes.byref(n)))
    return n.value


def hhg_mlp_set_params(m, params_f32):
    import numpy as np
    a = np.ascontiguousarray(params_f32, dtype=np.float32)
    _check(load().hhg_mlp_set_params(m, a.ctypes.data))


def hhg_mlp_get_params(m):
    import numpy as np
    a = np.empty(hhg_mlp_num_params(m), dtype=np.float32)
    _check(load().hhg_mlp_get_params(m, a.ctypes.data))
    return a


def hhg_mlp_forward(m, x, batch, y):
    _check(load().hhg_mlp_forward(m, _ptr(x), batch, _ptr(y)))


def hhg_mlp_loss_grad(m, x, y, batch):
    import numpy as np
    g = np.empty(hhg_mlp_num_params(m), dtype=np.float32)
    loss = ctypes.c_double()
    _check(load().hhg_mlp_loss_grad(m, _ptr(x), _ptr(y), batch, g.ctypes.data, ctypes.byref(loss)))
    return loss.value, g


def hhg_mlp_train(m, x, y, n_samples, batch, epochs, lr, order):
    import numpy as np
    o = np.ascontiguousarray(order, dtype=np.int32)
    loss = ctypes.c_double()
    _check(load().hhg_mlp_train(m, _ptr(x), _ptr(y), n_samples, batch, epochs, float(lr), o.ctypes.data,
                                ctypes.byref(loss)))
    return loss.value


def hhg_mlp_train_noalloc(m, x, y, n_samples, batch, epochs, lr, order):
    import numpy as np
    o = np.ascontiguousarray(order, dtype=np.int32)
    loss = ctypes.c_double()
    _check(load().hhg_mlp_train_noalloc(m, _ptr(x), _ptr(y), n_samples, batch, epochs, float(lr), o.ctypes.data,
                                        ctypes.byref(loss)))
    return loss.value


def hhg_mlp_dims(h):
    a, b = ctypes.c_int(), ctypes.c_int()
    _check(load().hhg_mlp_dims(h, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def hhg_coarse_pair(h, r, features, target):
    _check(load().hhg_coarse_pair(h, _ptr(r), _ptr(features), _ptr(target)))


def hhg_hier_set_fused_sites(h, max_sites):
    _check(load().hhg_hier_set_fused_sites(h, int(max_sites)))


def hhg_hier_set_bf16_levels(h, n):
    _check(load().hhg_hier_set_bf16_levels(h, n))


def hhg_record_pairs(h, features, targets, capacity):
    _check(load().hhg_record_pairs(h, _ptr(features) if capacity else None, _ptr(targets) if capacity else None,
                                   capacity))


def hhg_recorded_pairs(h):
    n = ctypes.c_int()
    _check(load().hhg_recorded_pairs(h, ctypes.byref(n)))
    return n.value


def hhg_hier_set_mlp(h, m, rho_plain=1.0, tau=0.0):
    _check(load().hhg_hier_set_mlp(h, m, float(rho_plain), float(tau)))
