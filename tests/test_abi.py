"""C-ABI checks that need no GPU: the library loads, exports every function
include/nsk.h declares, and nsk_create (host only) validates its input."""
import ctypes as C
import os
import re

import pytest

from paper_1912_12059_amd import nsk

HDR_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")


def _declared():
    names = set()
    for fn in os.listdir(HDR_DIR):
        if fn.endswith(".h"):
            txt = open(os.path.join(HDR_DIR, fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(nsk_\w+)\s*\(", txt))
    return sorted(names)


def test_every_declared_symbol_is_exported():
    lib = C.CDLL(nsk.LIB_PATH)
    names = _declared()
    assert "nsk_rk_step" in names and "nsk_create" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_names_match_header():
    for n in _declared():
        assert hasattr(nsk, n), f"binding lacks {n}"


def _ok_mesh(dim=3, N=4, nel=(4, 3, 2)):
    return nsk.make_mesh(dim, N, nel)


def test_create_sizes():
    m, keep = _ok_mesh()
    ctx = nsk.nsk_create(m, nsk.make_params())
    try:
        assert nsk.nsk_state_size(ctx) == 5 * 24 * 125
        assert nsk.nsk_workspace_bytes(ctx) >= 8 * (5 + 9) * 24 * 125
        m2, _ = nsk.make_mesh(2, 3, (5, 6))
        ctx2 = nsk.nsk_create(m2, nsk.make_params(precision=1))
        assert nsk.nsk_state_size(ctx2) == 4 * 30 * 16
        nsk.nsk_destroy(ctx2)
    finally:
        nsk.nsk_destroy(ctx)


@pytest.mark.parametrize("bad", [
    dict(dim=0), dict(dim=4), dict(N=0), dict(N=7), dict(nel=(0, 3, 2)), dict(nel=(4, -1, 2)),
])
def test_create_rejects_bad_mesh(bad):
    kw = dict(dim=3, N=4, nel=(4, 3, 2))
    kw.update(bad)
    m, keep = nsk.make_mesh(**kw)
    with pytest.raises(nsk.NskError) as e:
        nsk.nsk_create(m, nsk.make_params())
    assert e.value.code == nsk.NSK_EINVAL


@pytest.mark.parametrize("bad", [
    dict(T=0.0), dict(T=1.0), dict(alpha=0.0), dict(alpha=0.9), dict(T=0.5, alpha=2.9), dict(beta=0.0), dict(beta=-1.0), dict(eps=-1e-3),
    dict(kappa=-1.0), dict(precision=2), dict(flux=2), dict(closure=2), dict(diss_c=2),
    dict(alpha=float("nan")),
])
def test_create_rejects_bad_params(bad):
    m, keep = _ok_mesh()
    with pytest.raises(nsk.NskError) as e:
        nsk.nsk_create(m, nsk.make_params(**bad))
    assert e.value.code == nsk.NSK_EINVAL


def test_3d_degree_6_unsupported():
    m, keep = nsk.make_mesh(3, 6, (2, 2, 2))
    with pytest.raises(nsk.NskError) as e:
        nsk.nsk_create(m, nsk.make_params())
    assert e.value.code == nsk.NSK_EUNSUPPORTED


def test_create_rejects_bad_breakpoints():
    m, keep = nsk.make_mesh(1, 3, (3,), xbreaks=[[0.0, 0.5, 0.4, 1.0]])
    with pytest.raises(nsk.NskError):
        nsk.nsk_create(m, nsk.make_params())


def test_unbound_calls_fail_cleanly():
    m, keep = _ok_mesh()
    ctx = nsk.nsk_create(m, nsk.make_params())
    try:
        for fn, args in ((nsk.nsk_rk_step, (1e-6, 1)), (nsk.nsk_dt_estimate, (0.5,)),
                         (nsk.nsk_set_state, (1,)), (nsk.nsk_get_state, (1,))):
            with pytest.raises(nsk.NskError) as e:
                fn(ctx, *args)
            assert e.value.code == nsk.NSK_EUNBOUND
        with pytest.raises(nsk.NskError):
            nsk.nsk_rk_step(ctx, -1.0, 1)
    finally:
        nsk.nsk_destroy(ctx)


def test_rhs_noalloc_host_side_checks():
    """nsk_rhs_noalloc refuses, before any device call, problems whose
    gradients and geometry exceed its static scratch, the options it does not
    cover, and bad pointers."""
    big, keep = nsk.make_mesh(3, 4, (64, 64, 64))  # 32.8M nodes: 2.4 GB of FP64 gradients
    ctx = nsk.nsk_create(big, nsk.make_params())
    small, keep2 = _ok_mesh()
    ok = nsk.nsk_create(small, nsk.make_params())
    nub, keep3 = nsk.make_mesh(1, 3, (3,), xbreaks=[[0.0, 0.3, 0.5, 1.0]])
    nonuni = nsk.nsk_create(nub, nsk.make_params())
    sc = nsk.nsk_create(small, nsk.make_params(subcell=1, subcell_threshold=-9.0))
    try:
        with pytest.raises(nsk.NskError) as e:
            nsk.nsk_rhs_noalloc(ctx, 8, 16)
        assert e.value.code == nsk.NSK_ESCRATCH and "scratch" in nsk.nsk_strerror(nsk.NSK_ESCRATCH)
        for c in (nonuni, sc):
            with pytest.raises(nsk.NskError) as e:
                nsk.nsk_rhs_noalloc(c, 8, 16)
            assert e.value.code == nsk.NSK_EUNSUPPORTED
        for args in ((0, 16), (8, 0), (8, 8)):
            with pytest.raises(nsk.NskError) as e:
                nsk.nsk_rhs_noalloc(ok, *args)
            assert e.value.code == nsk.NSK_EINVAL
    finally:
        for c in (ctx, ok, nonuni, sc):
            nsk.nsk_destroy(c)


def test_closure_run_host_side_checks():
    """nsk_closure_run validates its two contexts and arguments on the host
    before touching a device."""
    m, keep = _ok_mesh()
    m2, keep2 = _ok_mesh(nel=(4, 3, 3))
    cl = nsk.nsk_create(m, nsk.make_params(alpha=200.0, closure=1))
    cl_nonet = nsk.nsk_create(m, nsk.make_params(alpha=200.0, closure=1))
    ref = nsk.nsk_create(m, nsk.make_params(alpha=2000.0))
    ref_other = nsk.nsk_create(m2, nsk.make_params(alpha=2000.0))
    ref_cl = nsk.nsk_create(m, nsk.make_params(alpha=2000.0, closure=1))
    norm = dict(s0=1.0, k0=1.0, s1=1.0, k1=1.0, k2=1.0, k3=1.0, g0=0.1, out_m=1.0, out_c=1.0)
    try:
        nsk.nsk_closure_set(cl, 256, norm, 1)  # a device address, never read by the checks
        nsk.nsk_closure_set(ref_cl, 256, norm, 1)
        bad = [(cl_nonet, ref, 1e-6, 4, 2, 2), (ref, ref, 1e-6, 4, 2, 2), (cl, ref_other, 1e-6, 4, 2, 2),
               (cl, ref_cl, 1e-6, 4, 2, 2), (cl, cl, 1e-6, 4, 2, 2), (cl, ref, 0.0, 4, 2, 2),
               (cl, ref, float("nan"), 4, 2, 2), (cl, ref, 1e-6, -1, 2, 2), (cl, ref, 1e-6, 4, 0, 2),
               (cl, ref, 1e-6, 4, 2, 0)]
        for args in bad:
            with pytest.raises(nsk.NskError) as e:
                nsk.nsk_closure_run(*args)
            assert e.value.code == nsk.NSK_EINVAL, args
        with pytest.raises(nsk.NskError) as e:
            nsk.nsk_closure_run(cl, ref, 1e-6, 4, 2, 2, float("inf"))
        assert e.value.code == nsk.NSK_EINVAL
        with pytest.raises(nsk.NskError) as e:
            nsk.nsk_closure_run(cl, ref, 1e-6, 4, 2, 2)
        assert e.value.code == nsk.NSK_EUNBOUND
    finally:
        for c in (cl, cl_nonet, ref, ref_other, ref_cl):
            nsk.nsk_destroy(c)


def test_strerror():
    assert "invalid" in nsk.nsk_strerror(nsk.NSK_EINVAL)
    assert nsk.nsk_strerror(12345) == "unknown error"


def test_closure_host_side_checks():
    """Closure entry points validate on the host before touching a device."""
    m, keep = _ok_mesh()
    plain = nsk.nsk_create(m, nsk.make_params(alpha=200.0))
    cl = nsk.nsk_create(m, nsk.make_params(alpha=200.0, closure=1))
    norm = dict(s0=1.0, k0=1.0, s1=1.0, k1=1.0, k2=1.0, k3=1.0, g0=0.1, out_m=1.0, out_c=1.0)
    try:
        # a closure context carries its FP32 source buffer in the workspace
        assert nsk.nsk_workspace_bytes(cl) > nsk.nsk_workspace_bytes(plain)
        fake = 256  # never dereferenced: every call below fails its host checks
        with pytest.raises(nsk.NskError):
            nsk.nsk_closure_set(plain, fake, norm)          # closure not enabled
        with pytest.raises(nsk.NskError):
            nsk.nsk_closure_set(cl, fake, dict(norm, g0=0.0))
        with pytest.raises(nsk.NskError):
            nsk.nsk_closure_set(cl, fake, dict(norm, k2=float("inf")))
        with pytest.raises(nsk.NskError):
            nsk.nsk_closure_set(cl, fake, norm, 2)  # every_stage must be 0 or 1
        # the parameters are staged 16 bytes at a time: a misaligned pointer
        # is refused, an aligned one accepted (it is only stored)
        with pytest.raises(nsk.NskError) as e:
            nsk.nsk_closure_set(cl, fake + 2, norm)
        assert e.value.code == nsk.NSK_EINVAL
        nsk.nsk_closure_set(cl, fake, norm)
        with pytest.raises(nsk.NskError) as e:
            nsk.nsk_mlp_forward(fake + 8, 0, 0, 0, 0)
        assert e.value.code == nsk.NSK_EINVAL
        nsk.nsk_mlp_forward(fake, 0, 0, 0, 0)  # nothing to do
        with pytest.raises(nsk.NskError) as e:
            nsk.nsk_closure_nudge(cl, norm, fake, 1e-6, 1e-4, 10.0, 0, 0)
        assert e.value.code == nsk.NSK_EUNBOUND
        with pytest.raises(nsk.NskError):
            nsk.nsk_closure_nudge(cl, norm, fake, 1e-6, 0.0, 10.0, 0, 0)  # tau <= 0
        # the closure flag fixes the workspace layout
        with pytest.raises(nsk.NskError):
            nsk.nsk_set_params(plain, nsk.make_params(alpha=200.0, closure=1))
        with pytest.raises(nsk.NskError):
            nsk.nsk_mlp_adam(fake, fake, fake, fake, fake, 0, 1e-3, 0.9, 0.999, 1e-8, 0)  # step 0
        with pytest.raises(nsk.NskError):
            nsk.nsk_mlp_loss_grad(fake, fake, fake, 0, 0, 1.0, 1.0, fake, fake, 0, 0)  # no samples
        nsk.nsk_mlp_forward(fake, fake, 0, fake, 0)  # nothing to do
        assert nsk.nsk_mlp_workspace_bytes(32768) >= 1024 * 8771 * 4
        bm, bkeep = nsk.make_mesh(3, 3, (2, 2, 2))
        with pytest.raises(nsk.NskError) as e:
            nsk.nsk_batch_create([bm], nsk.make_params(alpha=200.0, closure=1))
        assert e.value.code == nsk.NSK_EUNSUPPORTED
    finally:
        nsk.nsk_destroy(plain)
        nsk.nsk_destroy(cl)


def test_nsk_model_host_side_checks():
    """Original NSK path (model 1): state (rho, rho v), global Lax-Friedrichs
    flux only, FP64 only, no closure, alpha and beta unused; the batched form
    and the parameter changes that alter the workspace layout are refused."""
    m, keep = _ok_mesh()
    p = nsk.make_params(model=1, alpha=0.0, beta=0.0)
    assert p.flux == 2
    ctx = nsk.nsk_create(m, p)
    try:
        assert nsk.nsk_state_size(ctx) == 4 * 24 * 125
        plain = nsk.nsk_create(m, nsk.make_params())
        # the LF speed and its per-workgroup partial maxima live in the workspace
        assert nsk.nsk_workspace_bytes(ctx) >= 8 * (24 + 1)
        nsk.nsk_destroy(plain)
        with pytest.raises(nsk.NskError):
            nsk.nsk_set_params(ctx, nsk.make_params())  # model 0: other state layout
        nsk.nsk_set_params(ctx, nsk.make_params(model=1, eps=2e-3, kappa=1e-4))
    finally:
        nsk.nsk_destroy(ctx)
    for bad in (dict(flux=0), dict(flux=1), dict(precision=1), dict(closure=1), dict(kappa=-1.0),
                dict(eps=float("nan"))):
        q = nsk.make_params(model=1)
        for k, v in bad.items():
            setattr(q, k, v)
        with pytest.raises(nsk.NskError) as e:
            nsk.nsk_create(m, q)
        assert e.value.code == nsk.NSK_EINVAL, bad
    q = nsk.make_params()
    q.model = 2
    with pytest.raises(nsk.NskError):
        nsk.nsk_create(m, q)
    q = nsk.make_params(flux=2)  # the global LF flux is not a model II flux
    with pytest.raises(nsk.NskError):
        nsk.nsk_create(m, q)
    bm, bkeep = nsk.make_mesh(3, 3, (2, 2, 2))
    with pytest.raises(nsk.NskError) as e:
        nsk.nsk_batch_create([bm], nsk.make_params(model=1))
    assert e.value.code == nsk.NSK_EUNSUPPORTED


def test_implicit_host_side_checks():
    """nsk_esdirk_step validates its arguments on the host, before any device
    work: options, alignment, context kind, binding."""
    m, keep = _ok_mesh()
    ctx = nsk.nsk_create(m, nsk.make_params())
    mixed = nsk.nsk_create(m, nsk.make_params(precision=1))
    orig = nsk.nsk_create(m, nsk.make_params(model=1))
    try:
        M = 5 * 24 * 125
        assert nsk.nsk_implicit_workspace_bytes(ctx, 0) == 0
        assert nsk.nsk_implicit_workspace_bytes(ctx, nsk.NSK_GMRES_MAX + 1) == 0
        assert nsk.nsk_implicit_workspace_bytes(ctx, 20) >= 8 * (13 + 20 + 1) * M
        fake = 256  # never dereferenced: every call below fails its host checks
        ok = nsk.make_implicit_opts()
        for bad in (dict(newton_tol=0.0), dict(newton_max=0), dict(gmres_rtol=1.0), dict(gmres_rtol=0.0),
                    dict(gmres_m=0), dict(gmres_m=nsk.NSK_GMRES_MAX + 1), dict(precond=2), dict(basis_fp32=2),
                    dict(reorth_tol=-0.1), dict(reorth_tol=1.0)):
            with pytest.raises(nsk.NskError) as e:
                nsk.nsk_esdirk_step(ctx, fake, 1e-3, 1, nsk.make_implicit_opts(**bad))
            assert e.value.code == nsk.NSK_EINVAL, bad
        with pytest.raises(nsk.NskError) as e:
            nsk.nsk_esdirk_step(ctx, fake, -1.0, 1, ok)
        assert e.value.code == nsk.NSK_EINVAL
        with pytest.raises(nsk.NskError) as e:
            nsk.nsk_esdirk_step(ctx, fake + 8, 1e-3, 1, ok)  # not 256-byte aligned
        assert e.value.code == nsk.NSK_EINVAL
        with pytest.raises(nsk.NskError) as e:
            nsk.nsk_esdirk_step(mixed, fake, 1e-3, 1, ok)
        assert e.value.code == nsk.NSK_EUNSUPPORTED
        scx = nsk.nsk_create(m, nsk.make_params(subcell=1, subcell_threshold=-3.0))
        with pytest.raises(nsk.NskError) as e:
            nsk.nsk_esdirk_step(scx, fake, 1e-3, 1, ok)
        assert e.value.code == nsk.NSK_EUNSUPPORTED
        nsk.nsk_destroy(scx)
        with pytest.raises(nsk.NskError) as e:
            nsk.nsk_esdirk_step(orig, fake, 1e-3, 1, nsk.make_implicit_opts(precond=1))
        assert e.value.code == nsk.NSK_EINVAL
        with pytest.raises(nsk.NskError) as e:
            nsk.nsk_esdirk_step(ctx, fake, 1e-3, 1, ok)
        assert e.value.code == nsk.NSK_EUNBOUND
        assert "converge" in nsk.nsk_strerror(nsk.NSK_ENOCONV)
    finally:
        for c in (ctx, mixed, orig):
            nsk.nsk_destroy(c)


def test_subcell_host_side_checks():
    """FV sub-cells: model II with the Rusanov flux in FP64 without the
    closure only; the flags call needs a sub-cell context; the workspace
    holds the flags and the sub-cell means."""
    m, keep = _ok_mesh()
    plain = nsk.nsk_create(m, nsk.make_params())
    sc = nsk.nsk_create(m, nsk.make_params(subcell=1, subcell_threshold=-3.0))
    try:
        # flags, the needed-element marks and the sub-cell means (a state's worth)
        assert nsk.nsk_workspace_bytes(sc) >= nsk.nsk_workspace_bytes(plain) + 8 * 5 * 24 * 125
        with pytest.raises(nsk.NskError) as e:
            nsk.nsk_subcell_flags(plain, 256)
        assert e.value.code == nsk.NSK_EINVAL
        with pytest.raises(nsk.NskError) as e:
            nsk.nsk_subcell_flags(sc, 256)  # not bound yet
        assert e.value.code == nsk.NSK_EUNBOUND
        with pytest.raises(nsk.NskError):
            nsk.nsk_set_params(sc, nsk.make_params())  # the sub-cell workspace is part of the layout
    finally:
        nsk.nsk_destroy(plain)
        nsk.nsk_destroy(sc)
    for bad in (dict(flux=2), dict(precision=1), dict(closure=1), dict(subcell=2),
                dict(subcell_threshold=float("nan")), dict(model=1, flux=2)):
        kw = dict(subcell=1, subcell_threshold=-3.0)
        kw.update(bad)
        with pytest.raises(nsk.NskError) as e:
            nsk.nsk_create(m, nsk.make_params(**kw))
        assert e.value.code == nsk.NSK_EINVAL, bad
    bm, bkeep = nsk.make_mesh(3, 3, (2, 2, 2))
    with pytest.raises(nsk.NskError) as e:
        nsk.nsk_batch_create([bm], nsk.make_params(subcell=1, subcell_threshold=-3.0))
    assert e.value.code == nsk.NSK_EUNSUPPORTED
    # the batch kernels are instantiated for the Rusanov flux only
    with pytest.raises(nsk.NskError) as e:
        nsk.nsk_batch_create([bm], nsk.make_params(flux=1))
    assert e.value.code == nsk.NSK_EUNSUPPORTED


def test_core_host_side_checks():
    """Argument and binding checks of the core entry points, taken before any
    device work (the pointers below are never dereferenced)."""
    m, keep = _ok_mesh()
    ctx = nsk.nsk_create(m, nsk.make_params())
    fake_u, fake_r = 0x1000, 0x2000
    try:
        # launch shape: 2 variants x 6 orders; an unbound context only stores it
        for v, o in ((-1, 0), (2, 0), (0, -1), (0, 6)):
            with pytest.raises(nsk.NskError) as e:
                nsk.nsk_set_tile(ctx, v, o)
            assert e.value.code == nsk.NSK_EINVAL
        nsk.nsk_set_tile(ctx, 1, 5)
        with pytest.raises(nsk.NskError) as e:
            nsk.nsk_autotune(ctx, 0)
        assert e.value.code == nsk.NSK_EINVAL
        with pytest.raises(nsk.NskError) as e:
            nsk.nsk_autotune(ctx, 3)
        assert e.value.code == nsk.NSK_EUNBOUND
        # rhs: output aliasing the input, null pointers, then the binding
        for u, r in ((fake_u, fake_u), (0, fake_r), (fake_u, 0)):
            with pytest.raises(nsk.NskError) as e:
                nsk.nsk_rhs(ctx, u, r)
            assert e.value.code == nsk.NSK_EINVAL
        with pytest.raises(nsk.NskError) as e:
            nsk.nsk_rhs(ctx, fake_u, fake_r)
        assert e.value.code == nsk.NSK_EUNBOUND
        with pytest.raises(nsk.NskError) as e:
            nsk.nsk_diagnostics(ctx)
        assert e.value.code == nsk.NSK_EUNBOUND
        # sub-cell flags exist only in sub-cell contexts
        with pytest.raises(nsk.NskError) as e:
            nsk.nsk_subcell_flags(ctx, fake_u)
        assert e.value.code == nsk.NSK_EINVAL
        # the workspace layout fixes model, precision, closure and sub-cell flag
        for kw in (dict(precision=1), dict(model=1, flux=2), dict(subcell=1)):
            with pytest.raises(nsk.NskError) as e:
                nsk.nsk_set_params(ctx, nsk.make_params(**kw))
            assert e.value.code == nsk.NSK_EINVAL
        nsk.nsk_set_params(ctx, nsk.make_params(alpha=800.0))
        # nothing timed yet: zeros
        assert nsk.nsk_timing_read(ctx) == (0.0, 0.0, 0, 0.0)
    finally:
        nsk.nsk_destroy(ctx)


def test_batch_host_side_checks():
    """Packing of the batched state and the batch entry points' argument and
    binding checks, before any device work."""
    m1, k1 = nsk.make_mesh(3, 3, (4, 3, 2))
    m2, k2 = nsk.make_mesh(3, 4, (3, 3, 3))
    b = nsk.nsk_batch_create([m1, m2], nsk.make_params())
    try:
        # instance slices: in order, disjoint, 256-byte aligned
        n0, n1 = 5 * 24 * 64, 5 * 27 * 125
        o0, o1 = nsk.nsk_batch_state_offset(b, 0), nsk.nsk_batch_state_offset(b, 1)
        assert o0 == 0 and o1 >= o0 + n0 and o1 % 32 == 0
        assert nsk.nsk_batch_state_size(b) >= o1 + n1
        assert [g["N"] for g in nsk.nsk_batch_groups(b)] == [3, 4]
        assert nsk.nsk_batch_ctx(b, 1) != 0
        for inst in (-1, 2):
            with pytest.raises(nsk.NskError) as e:
                nsk.nsk_batch_ctx(b, inst)
            assert e.value.code == nsk.NSK_EINVAL
        # group launch shapes: group index, variant, grid multiple, order, chunk
        for args in ((2, 0, 0, 0, 0), (0, 2, 0, 0, 0), (0, 0, 3, 0, 0), (0, 0, 0, 6, 0), (0, 0, 0, 0, -1)):
            with pytest.raises(nsk.NskError) as e:
                nsk.nsk_batch_set_group(b, *args)
            assert e.value.code == nsk.NSK_EINVAL
        with pytest.raises(nsk.NskError) as e:
            nsk.nsk_batch_set_group(b, 1, 1, 4, 3, 8)
        assert e.value.code == nsk.NSK_EUNBOUND
        for bad_dt in (0.0, -1e-6, float("nan"), float("inf")):
            with pytest.raises(nsk.NskError) as e:
                nsk.nsk_batch_rk_step(b, bad_dt, 1)
            assert e.value.code == nsk.NSK_EINVAL
        for fn, args in ((nsk.nsk_batch_rk_step, (1e-6, 2)), (nsk.nsk_batch_dt_estimate, (0.5,)),
                         (nsk.nsk_batch_autotune, (2,))):
            with pytest.raises(nsk.NskError) as e:
                fn(b, *args)
            assert e.value.code == nsk.NSK_EUNBOUND
        # only 3D instances
        m3, k3 = nsk.make_mesh(2, 4, (5, 5))
        with pytest.raises(nsk.NskError) as e:
            nsk.nsk_batch_create([m1, m3], nsk.make_params())
        assert e.value.code == nsk.NSK_EUNSUPPORTED
    finally:
        nsk.nsk_batch_destroy(b)
