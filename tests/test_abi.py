"""The C-ABI library loads, exports every symbol its header declares, and
rejects bad arguments on the host before any HIP call (so these run
without a GPU: no call here reaches a kernel launch)."""

import ctypes
import os
import re

import pytest

from paper_2312_06827_amd import lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sv.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sv_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def so():
    if not os.path.exists(L.LIB_PATH):
        pytest.fail("libsv.so is not built (run __graft_entry__.build())")
    return L.load()


def test_every_declared_symbol_is_exported(so):
    names = declared_functions()
    assert {"sv_tonemap", "sv_clamp", "sv_temporal", "sv_variance", "sv_atrous",
            "sv_atrous_sep"} <= set(names)
    for n in names:
        assert hasattr(so, n), n
    assert set(names) <= set(L.EXPORTS)


def test_status_strings_and_version(so):
    assert so.sv_version() == 1
    for code in range(7):
        assert so.sv_status_str(code)
    assert so.sv_status_str(99) == b"unknown status"
    assert so.sv_last_hip_error() == 0


# Fake device addresses: never dereferenced, every case below fails
# validation before a launch.
A = 0x10000000
STRIDE = 0x01000000


def rgb(base):
    return L.sv_rgb(base, base + STRIDE, base + 2 * STRIDE)


def gbuf(base):
    return L.sv_gbuf(*[base + i * STRIDE for i in range(6)], None)


D = L.sv_dims(64, 32, 64)
TM = L.sv_tm_params(1.0, 1.0, L.SV_TM_LUMA)
AP = L.sv_atrous_params(1.0, 128.0, 4.0, 1e-10, 1e-10, 1.0, 0, -1, 0)


def test_tonemap_validation(so):
    r = ctypes.byref
    assert so.sv_tonemap(None, r(rgb(A)), D, L.SV_F32, 0, r(TM), None) == L.SV_EINVAL
    assert so.sv_tonemap(r(rgb(A)), r(rgb(A)), D, 7, 0, r(TM), None) == L.SV_EDTYPE
    assert so.sv_tonemap(r(rgb(A)), r(rgb(A)), L.sv_dims(64, 32, 10), L.SV_F32, 0, r(TM),
                         None) == L.SV_EINVAL
    assert so.sv_tonemap(r(rgb(A)), r(rgb(A)), L.sv_dims(-1, 32, 64), L.SV_F32, 0, r(TM),
                         None) == L.SV_EINVAL
    paper_fwd = L.sv_tm_params(1.0, 1.0, L.SV_TM_PAPER)
    assert so.sv_tonemap(r(rgb(A)), r(rgb(A)), D, L.SV_F32, 0, r(paper_fwd),
                         None) == L.SV_EUNSUPPORTED
    # empty image: valid, nothing enqueued
    assert so.sv_tonemap(r(rgb(A)), r(rgb(A)), L.sv_dims(0, 32, 64), L.SV_F32, 0, r(TM),
                         None) == L.SV_OK
    big = L.sv_dims(32768, 32768, 65536)
    assert so.sv_tonemap(r(rgb(A)), r(rgb(A)), big, L.SV_F32, 0, r(TM), None) == L.SV_EINVAL
    # the limits: pitch * h <= 2^29 elements, w and h <= 32768
    over = L.sv_dims(64, 32768, 16385)  # one row's pitch over 2^29
    assert so.sv_tonemap(r(rgb(A)), r(rgb(A)), over, L.SV_F32, 0, r(TM), None) == L.SV_EINVAL
    for dims in (L.sv_dims(32769, 1, 32769), L.sv_dims(1, 32769, 1)):
        assert so.sv_tonemap(r(rgb(A)), r(rgb(A)), dims, L.SV_F32, 0, r(TM), None) == L.SV_EINVAL


def test_clamp_and_clip_validation(so):
    r = ctypes.byref
    B = A + 0x20000000
    for fn in (so.sv_clamp, so.sv_clip):
        assert fn(None, r(rgb(A)), r(rgb(B)), None, D, L.SV_F32, 1.0, None) == L.SV_EINVAL
        assert fn(r(rgb(A)), r(rgb(A)), r(rgb(B)), None, D, 5, 1.0, None) == L.SV_EDTYPE
        # the output on top of the current colour (the box's source)
        assert fn(r(rgb(A)), r(rgb(B)), r(rgb(B + 64)), None, D, L.SV_F32, 1.0,
                  None) == L.SV_EALIAS
        # or of the depth plane
        assert fn(r(rgb(A)), r(rgb(B)), r(rgb(A)), A + 4, D, L.SV_F32, 1.0,
                  None) == L.SV_EALIAS
        assert fn(r(rgb(A)), r(rgb(B)), r(rgb(A)), None, L.sv_dims(0, 4, 4), L.SV_F32, 1.0,
                  None) == L.SV_OK


def test_atrous_validation_and_aliasing(so):
    r = ctypes.byref
    B = A + 0x20000000
    g = gbuf(A + 0x40000000)
    var = A + 0x60000000
    # step must be >= 1
    assert so.sv_atrous(r(rgb(A)), var, r(g), None, r(rgb(B)), None, 0, D, L.SV_F32, r(AP),
                        None) == L.SV_EINVAL
    # output overlapping the input colour
    assert so.sv_atrous(r(rgb(A)), var, r(g), None, r(rgb(A + 64)), None, 1, D, L.SV_F32,
                        r(AP), None) == L.SV_EALIAS
    # output variance overlapping the G-buffer
    assert so.sv_atrous(r(rgb(A)), var, r(g), None, r(rgb(B)), A + 0x40000000 + 128, 1, D,
                        L.SV_F32, r(AP), None) == L.SV_EALIAS
    # two outputs on top of each other
    assert so.sv_atrous(r(rgb(A)), var, r(g), None, L.sv_rgb(B, B, B + STRIDE), None, 1, D,
                        L.SV_F32, r(AP), None) == L.SV_EALIAS
    # missing G-buffer plane
    g2 = gbuf(A + 0x40000000)
    g2.nz = None
    assert so.sv_atrous(r(rgb(A)), var, r(g2), None, r(rgb(B)), None, 1, D, L.SV_F32, r(AP),
                        None) == L.SV_EINVAL
    # without scratch (the fused form) only steps 1..32 are available; with
    # scratch, it must not alias the output
    assert so.sv_atrous_sep(r(rgb(A)), var, r(g), None, None, r(rgb(B)), None, 64, D, L.SV_F32,
                            r(AP), None) == L.SV_EUNSUPPORTED
    assert so.sv_atrous_sep(r(rgb(A)), var, r(g), None, L.sv_rgb(B, None, B), r(rgb(B)), None,
                            1, D, L.SV_F32, r(AP), None) == L.SV_EINVAL
    assert so.sv_atrous_sep(r(rgb(A)), var, r(g), None, r(rgb(B)), r(rgb(B)), None, 1, D,
                            L.SV_F32, r(AP), None) == L.SV_EALIAS
    bad = L.sv_atrous_params(1.0, -1.0, 4.0, 1e-10, 1e-10, 1.0, 0, -1, 0)
    assert so.sv_atrous(r(rgb(A)), var, r(g), None, r(rgb(B)), None, 1, D, L.SV_F32, r(bad),
                        None) == L.SV_EINVAL


def test_temporal_and_variance_validation(so):
    r = ctypes.byref
    io = L.sv_temporal_io()
    p = L.sv_temporal_params(0.2, 0.2, 1.0, 0.1, 0.9, 1.0, 255, 0)
    assert so.sv_temporal(r(io), D, L.SV_F32, r(p), None) == L.SV_EINVAL
    base = [A + i * 0x01000000 for i in range(40)]
    io = L.sv_temporal_io(rgb(base[0]), gbuf(base[3]), base[9], base[10], gbuf(base[11]),
                          rgb(base[17]), base[20], base[21], base[22], rgb(base[23]),
                          base[26], base[27], base[28], None)
    # clamp and clip together
    both = L.sv_temporal_params(0.2, 0.2, 1.0, 0.1, 0.9, 1.0, 255, L.SV_T_CLAMP | L.SV_T_CLIP)
    assert so.sv_temporal(r(io), D, L.SV_F32, r(both), None) == L.SV_EINVAL
    # output moments on top of the history moments
    io.out_m1 = base[20]
    assert so.sv_temporal(r(io), D, L.SV_F32, r(p), None) == L.SV_EALIAS
    io.out_m1 = base[26]
    p_bad = L.sv_temporal_params(0.2, 0.2, 1.0, 0.1, 0.9, 1.0, 0, 0)
    assert so.sv_temporal(r(io), D, L.SV_F32, r(p_bad), None) == L.SV_EINVAL
    p_id = L.sv_temporal_params(0.2, 0.2, 1.0, 0.1, 0.9, 1.0, 255, L.SV_T_USE_ID)
    assert so.sv_temporal(r(io), D, L.SV_F32, r(p_id), None) == L.SV_EINVAL
    vp = L.sv_variance_params(1.0, 128.0, 1e-10, 4, 8)
    g = gbuf(base[3])
    assert so.sv_variance(base[30], base[31], base[32], r(g), base[33], base[34], D, L.SV_F32,
                          r(vp), None) == L.SV_EINVAL
    vp = L.sv_variance_params(1.0, 128.0, 1e-10, 4, 3)
    assert so.sv_variance(base[30], base[31], base[32], r(g), base[30], base[34], D, L.SV_F32,
                          r(vp), None) == L.SV_EALIAS
    # the workspace must not overlap an input
    assert so.sv_variance(base[30], base[31], base[32], r(g), base[33], base[31], D, L.SV_F32,
                          r(vp), None) == L.SV_EALIAS
    assert so.sv_variance(base[30], base[31], base[32], r(g), base[33], None, D, L.SV_F32,
                          r(vp), None) == L.SV_EINVAL
    assert so.sv_variance_work_bytes(D) == 1024 + 4 * 256 * 8  # 64x32: 8 tiles of 64x4
    assert so.sv_variance_work_bytes(L.sv_dims(-1, 2, 2)) == 0


def test_probe_copy_validation(so):
    assert so.sv_probe_copy(None, A, 64, None) == L.SV_EINVAL
    assert so.sv_probe_copy(A, A + 0x100000, 60, None) == L.SV_EINVAL
    assert so.sv_probe_copy(A, A + 32, 64, None) == L.SV_EALIAS
    assert so.sv_probe_copy(A, A + 0x100000, 0, None) == L.SV_OK


def test_issue_probe_validation(so):
    out = A
    assert so.sv_probe_issue(0, 16, None, 4, None) == L.SV_EINVAL
    for kind, iters, blocks in ((-1, 16, 4), (5, 16, 4), (0, 0, 4), (0, 1 << 21, 4), (0, 16, 0),
                                (0, 16, 65537)):
        assert so.sv_probe_issue(kind, iters, out, blocks, None) == L.SV_EINVAL


def test_binding_rejects_host_tensors():
    import torch
    t = torch.zeros((3, 4, 4))
    with pytest.raises(ValueError):
        L.sv_tonemap(t, t)


def test_mlp_validation(so):
    r = ctypes.byref
    base = [A + i * 0x01000000 for i in range(48)]
    w = L.sv_mlp(base[40], base[41], base[42], base[43])
    feat = base[44]
    # missing parameters, misaligned or missing feature rows
    assert so.sv_mlp_forward(r(L.sv_mlp(None, base[41], None, None)), feat, base[30], None, D,
                             None) == L.SV_EINVAL
    assert so.sv_mlp_forward(r(w), feat + 8, base[30], None, D, None) == L.SV_EINVAL
    assert so.sv_mlp_forward(r(w), None, base[30], None, D, None) == L.SV_EINVAL
    # outputs on top of the rows or of each other
    assert so.sv_mlp_forward(r(w), feat, feat + 64, None, D, None) == L.SV_EALIAS
    assert so.sv_mlp_forward(r(w), feat, base[30], base[30] + 4, D, None) == L.SV_EALIAS
    # backward: workspace, gradient and inputs must be distinct
    wb = so.sv_mlp_backward_work_bytes(D)
    # 2048 pixels = 64 blocks of 32, four per workgroup: 16 workgroups x 4 waves
    assert wb == 16 * 4 * L.SV_MLP_PARAMS * 4
    assert so.sv_mlp_backward(r(w), feat, base[30], base[31], 1.0, base[32], None, D,
                              None) == L.SV_EINVAL
    assert so.sv_mlp_backward(r(w), feat, base[30], base[31], 1.0, base[32], base[32] + 16, D,
                              None) == L.SV_EALIAS
    assert so.sv_mlp_backward(r(w), feat, base[30], base[31], 1.0, base[30], base[33], D,
                              None) == L.SV_EALIAS
    ap = L.sv_adam_params(1e-3, 0.9, 0.999, 1e-8)
    assert so.sv_adam(base[40], base[41], base[42], base[43], base[44], 10, 0, r(ap),
                      None) == L.SV_EINVAL
    assert so.sv_adam(None, None, base[42], base[43], base[44], 10, 1, r(ap), None) == L.SV_EINVAL
    # features: the history colour output must not overlap an input
    io = L.sv_temporal_io(rgb(base[0]), gbuf(base[3]), base[9], base[10], gbuf(base[11]),
                          rgb(base[17]), base[20], base[21], base[22], L.sv_rgb(), None, None,
                          None, None)
    p = L.sv_temporal_params(0.2, 0.2, 1.0, 0.1, 0.9, 1.0, 255, 0)
    assert so.sv_mlp_features(r(io), r(rgb(base[25])), r(w), feat, r(rgb(base[0])), D,
                              L.SV_F32, r(p), None) == L.SV_EALIAS
    assert so.sv_mlp_features(r(io), None, r(w), feat, None, D, L.SV_F32, r(p),
                              None) == L.SV_EINVAL
    assert so.sv_mlp_features(r(io), r(rgb(base[25])), r(w), feat + 4, None, D, L.SV_F32, r(p),
                              None) == L.SV_EINVAL
    # loss gradients
    assert so.sv_mlp_alpha_grad(r(rgb(base[0])), r(rgb(base[3])), r(rgb(base[6])),
                                r(rgb(base[9])), base[12], base[13], base[14], 1.0, base[12],
                                D, L.SV_F32, None) == L.SV_EALIAS
    g = gbuf(base[20])
    assert so.sv_atrous_kappa_grad(r(rgb(base[0])), base[3], r(g), base[4], r(rgb(base[5])),
                                   None, base[4], 1, D, L.SV_F32, r(AP), None) == L.SV_EALIAS
    assert so.sv_atrous_kappa_grad(r(rgb(base[0])), base[3], r(g), base[4], r(rgb(base[5])),
                                   None, base[8], 0, D, L.SV_F32, r(AP), None) == L.SV_EINVAL
    # the residual source must not overlap the gradient it accumulates into
    assert so.sv_atrous_kappa_grad(r(rgb(base[0])), base[3], r(g), base[4], r(rgb(base[5])),
                                   r(rgb(base[8])), base[9], 1, D, L.SV_F32, r(AP),
                                   None) == L.SV_EALIAS


def test_batch_validation(so):
    r = ctypes.byref
    out = ctypes.c_void_p()
    lp = (ctypes.c_int32 * 10)(*([-1] * 10))
    lb = (ctypes.c_int32 * 10)(*([0] * 10))
    tp = L.sv_temporal_params(0.2, 0.2, 1.0, 0.1, 0.9, 1.0, 255, 0)
    vp = L.sv_variance_params(1.0, 128.0, 1e-10, 4, 3)
    fp = L.sv_frame_params(tp, vp, AP, 5, 0, 0, lp, lb)
    st = [L.sv_denoiser(), L.sv_denoiser()]
    states = (ctypes.POINTER(L.sv_denoiser) * 2)(*[ctypes.pointer(x) for x in st])
    dims = (L.sv_dims * 2)(D, L.sv_dims(100, 20, 128))
    assert so.sv_batch_create(dims, states, 0, L.SV_F32, r(fp), r(out)) == L.SV_EINVAL
    assert so.sv_batch_create(dims, states, 2, 9, r(fp), r(out)) == L.SV_EDTYPE
    bad = (L.sv_dims * 2)(D, L.sv_dims(0, 20, 128))  # an empty stream
    assert so.sv_batch_create(bad, states, 2, L.SV_F32, r(fp), r(out)) == L.SV_EINVAL
    same = (ctypes.POINTER(L.sv_denoiser) * 2)(ctypes.pointer(st[0]), ctypes.pointer(st[0]))
    assert so.sv_batch_create(dims, same, 2, L.SV_F32, r(fp), r(out)) == L.SV_EALIAS
    fp6 = L.sv_frame_params(tp, vp, AP, 6, 0, 0, lp, lb)
    assert so.sv_batch_create(dims, states, 2, L.SV_F32, r(fp6), r(out)) == L.SV_EUNSUPPORTED
    fp1 = L.sv_frame_params(tp, vp, AP, 1, 0, 0, lp, lb)
    assert so.sv_batch_create(dims, states, 2, L.SV_F32, r(fp1), r(out)) == L.SV_EUNSUPPORTED
    # a valid plan: nothing is allocated until the first frame
    assert so.sv_batch_create(dims, states, 2, L.SV_F32, r(fp), r(out)) == L.SV_OK
    assert so.sv_batch_passes(out) == 0
    assert so.sv_batch_frame(out, None, None) == L.SV_EINVAL
    so.sv_batch_destroy(out)
    assert so.sv_batch_passes(None) == -1


def test_binding_structures_match_the_header(so):
    """Every ctypes structure of the binding has the C structure's size."""
    sizes = (ctypes.c_size_t * 32)()
    k = so.sv_struct_sizes(sizes, 32)
    mine = [L.sv_dims, L.sv_rgb, L.sv_gbuf, L.sv_tm_params, L.sv_temporal_io,
            L.sv_temporal_params, L.sv_variance_params, L.sv_atrous_params, L.sv_denoiser,
            L.sv_frame_in, L.sv_frame_params, L.sv_mlp, L.sv_adam_params, L.sv_blur_rule,
            L.sv_grad_params]
    assert k == len(mine)
    for i, t in enumerate(mine):
        assert ctypes.sizeof(t) == sizes[i], (t.__name__, ctypes.sizeof(t), sizes[i])


def test_variance_noalloc_rejects_on_the_host(so):
    """Sizes past the fixed 32 MiB workspace fail with SV_ETOOBIG, and the
    listed mode with SV_EINVAL, before any HIP call."""
    vp = L.sv_variance_params(1.0, 128.0, 1e-10, 4, 3, 0)
    r = ctypes.byref
    g = gbuf(A)
    big = L.sv_dims(4096, 2304, 4096)  # needs 37.7 MB of workspace
    assert so.sv_variance_work_bytes(big) > 32 << 20
    assert so.sv_variance_noalloc(A, A + STRIDE, A + 2 * STRIDE, r(g), A + 3 * STRIDE, big,
                                  L.SV_F32, r(vp), None) == L.SV_ETOOBIG
    uhd = L.sv_dims(3840, 2160, 3840)
    assert so.sv_variance_work_bytes(uhd) <= 32 << 20
    listed = L.sv_variance_params(1.0, 128.0, 1e-10, 4, 3, L.SV_V_LISTED)
    assert so.sv_variance_noalloc(A, A + STRIDE, A + 2 * STRIDE, r(g), A + 3 * STRIDE, uhd,
                                  L.SV_F32, r(listed), None) == L.SV_EINVAL
    empty = L.sv_dims(0, 10, 0)
    assert so.sv_variance_noalloc(None, None, None, r(g), None, empty, L.SV_F32, r(vp),
                                  None) == L.SV_OK


def test_gradient_validation(so):
    """The temporal gradient's workspace must be 16-byte aligned (its cell
    keys are 64-bit atomics, its cells float4); bad parameters and
    aliasing are refused before any HIP call."""
    r = ctypes.byref
    gp = L.sv_grad_params(0.2, 0.1, 1.0, 3)
    work = A + 20 * STRIDE
    args = lambda wk, p=gp: (r(rgb(A)), r(rgb(A + 3 * STRIDE)), A + 6 * STRIDE, A + 7 * STRIDE,
                             A + 8 * STRIDE, A + 9 * STRIDE, r(gbuf(A + 10 * STRIDE)),
                             A + 18 * STRIDE, None, wk, D, L.SV_F32, r(p), None)
    assert so.sv_grad_work_bytes(D) >= 22 * 11 * 8
    assert so.sv_temporal_gradient(*args(work + 8)) == L.SV_EINVAL
    assert so.sv_temporal_gradient(*args(work, L.sv_grad_params(0.2, 0.1, 1.0, 9))) == L.SV_EINVAL
    assert so.sv_temporal_gradient(*args(A + 8 * STRIDE)) == L.SV_EALIAS


def test_batch_set_direct_validation(so):
    assert so.sv_batch_set_direct(None, 0) == L.SV_EINVAL
    assert so.sv_batch_set_direct(None, 1) == L.SV_EINVAL
