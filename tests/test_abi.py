"""The C-ABI library loads and exports every function that include/veg.h declares (CPU)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "veg.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(veg_[a-z0-9_]+)\s*\(", text))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("veg_project", "veg_bin_count", "veg_bin_sort", "veg_render_fwd", "veg_render_bwd",
                     "veg_project_bwd", "veg_serve_create", "veg_serve_submit", "veg_serve_wait"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_2504_13339_amd as pkg
    lib = pkg.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", pkg.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (veg_\w+)", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing


def test_binding_declares_the_same_names():
    from paper_2504_13339_amd import _lib
    assert set(_lib.declared_symbols()) == set(declared_functions())


def test_host_side_argument_errors_without_gpu():
    """Argument validation happens before anything touches the device."""
    import ctypes
    from paper_2504_13339_amd import _lib
    lib = _lib.load()
    o = _lib.veg_opts()
    lib.veg_opts_default(ctypes.byref(o))
    assert abs(o.alpha_min - 1 / 255) < 1e-9 and abs(o.alpha_clamp - 0.99) < 1e-7
    assert lib.veg_project(None, 1, None, None, None, None, None) == 1
    assert lib.veg_l1_loss(None, None, -1, 1.0, None, None, None) == 1
    assert b"count" in lib.veg_last_error()
    assert lib.veg_fill_u32(None, 5, 0, None) == 1
    assert lib.veg_status_str(6) == b"HIP error"


def test_image_loss_arguments_are_checked_on_host():
    """veg_image_loss refuses bad sizes, NULL buffers, non-finite weights and a small
    workspace before anything is enqueued; an empty image is a no-op."""
    import ctypes
    from paper_2504_13339_amd import _lib
    lib = _lib.load()
    fake = ctypes.c_void_p(0x10000)
    f = ctypes.c_float
    need = lib.veg_ssim_workspace_bytes(2, 8, 8)
    assert lib.veg_image_loss(fake, fake, 70000, 8, 8, f(0.5), f(0.5), fake, fake, fake, need, None) == 1
    assert b"sizes" in lib.veg_last_error()
    assert lib.veg_image_loss(None, fake, 2, 8, 8, f(0.5), f(0.5), fake, fake, fake, need, None) == 1
    assert b"NULL" in lib.veg_last_error()
    assert lib.veg_image_loss(fake, fake, 2, 8, 8, f(float("nan")), f(0.5), fake, fake, fake, need, None) == 1
    assert b"finite" in lib.veg_last_error()
    assert lib.veg_image_loss(fake, fake, 2, 8, 8, f(0.5), f(0.5), fake, fake, fake, need - 4, None) == 1
    assert b"workspace" in lib.veg_last_error()
    assert lib.veg_image_loss(None, None, 0, 8, 8, f(0.5), f(0.5), None, None, None, 0, None) == 0


def test_bin_status_arguments_are_checked_on_host():
    """veg_bin_status rejects a missing or small workspace and a NULL or misaligned
    destination before any device call (host pointers stand in for device ones)."""
    import ctypes
    from paper_2504_13339_amd import _lib
    lib = _lib.load()
    nb = int(lib.veg_bin_workspace_bytes(1, 0))
    ws = (ctypes.c_uint8 * nb)()
    dst = (ctypes.c_int64 * 4)()
    base = ctypes.addressof(dst)
    assert lib.veg_bin_status(None, nb, base, None) == 1
    assert lib.veg_bin_status(ctypes.addressof(ws), 8, base, None) == 1
    assert b"workspace" in lib.veg_last_error()
    assert lib.veg_bin_status(ctypes.addressof(ws), nb, None, None) == 1
    assert lib.veg_bin_status(ctypes.addressof(ws), nb, base + 4, None) == 1
    assert b"misaligned" in lib.veg_last_error()


def test_serve_config_validation_on_host():
    import ctypes
    from paper_2504_13339_amd import _lib
    lib = _lib.load()
    cfg = _lib.veg_serve_config()
    cfg.max_batch, cfg.n_streams, cfg.max_width, cfg.max_height, cfg.max_tf_k = 8, 2, 1920, 1080, 256
    cfg.max_gaussians, cfg.max_entries = 3_000_000, 100_000_000
    need = lib.veg_serve_arena_bytes(ctypes.byref(cfg))
    # per slot: 88 B per pair (48 record, 8 count/depth, 32 bin workspace) + 16 B per key-list entry
    assert 2 * (24_000_000 * 88 + 100_000_000 * 16) <= need < 2 * (24_000_000 * 96 + 100_000_000 * 16) + (1 << 26)
    cfg.max_batch = 0
    assert lib.veg_serve_arena_bytes(ctypes.byref(cfg)) == 0
    cfg.max_batch = 8
    h = ctypes.c_void_p()
    assert lib.veg_serve_create(ctypes.byref(cfg), ctypes.byref(h)) == 1      # NULL arena
    assert b"arena" in lib.veg_last_error()


def test_hit_bits_buffer_is_validated_on_host():
    """A hit-bit buffer smaller than veg_bin_hit_words(capacity, tiles) is rejected before any
    launch (the pointers below are never dereferenced)."""
    import ctypes
    from paper_2504_13339_amd import _lib
    lib = _lib.load()
    assert lib.veg_bin_hit_words(64, 1) == 64 // 64 + 1 + 2
    assert lib.veg_bin_hit_words(1000, 4096 * 16) == 1000 // 64 + 4096 * 16 + 2
    fake = ctypes.c_void_p(0x10000)
    p = _lib.veg_proj(1, 1, 16, 16, 1, 1, 1, fake, fake, fake, fake)
    b = _lib.veg_bins(fake, fake, fake, fake, fake, 64, fake, 3)
    img = ctypes.c_void_p(0x20000)
    assert lib.veg_render_fwd(ctypes.byref(p), ctypes.byref(b), None, img, None, None, None, None) == 1
    assert b"hit_words" in lib.veg_last_error()
    assert lib.veg_render_bwd(ctypes.byref(p), ctypes.byref(b), None, img, img, img, img, None) == 1
    assert b"hit_words" in lib.veg_last_error()


def test_shared_view_hit_bits_and_frame_grouping_on_host():
    """With tfs_per_view = K the hit-bit buffer needs K blocks of veg_bin_hit_words, and the
    frame count must be a multiple of K (checked before any launch)."""
    import ctypes
    from paper_2504_13339_amd import _lib
    lib = _lib.load()
    fake = ctypes.c_void_p(0x10000)
    img = ctypes.c_void_p(0x20000)
    stride = lib.veg_bin_hit_words(64, 1)           # one list of one tile for the three frames
    p = _lib.veg_proj(1, 3, 16, 16, 1, 1, 1, fake, fake, fake, fake, 3)
    b = _lib.veg_bins(fake, fake, fake, fake, fake, 64, fake, 3 * stride - 1)
    assert lib.veg_render_fwd(ctypes.byref(p), ctypes.byref(b), None, img, None, None, None, None) == 1
    assert b"tfs_per_view" in lib.veg_last_error()
    p2 = _lib.veg_proj(1, 4, 16, 16, 1, 1, 1, fake, fake, fake, fake, 3)
    assert lib.veg_render_bwd(ctypes.byref(p2), ctypes.byref(b), None, img, img, img, img, None) == 1
    assert b"multiple" in lib.veg_last_error()


def test_views_of_detects_view_major_products():
    from paper_2504_13339_amd import render as R
    assert R.views_of([(0, 0), (0, 1), (1, 0), (1, 1)]) == 2
    assert R.views_of([(0, 0), (1, 0)]) == 1
    assert R.views_of([(0, 0), (0, 1), (1, 1), (1, 0)]) == 0
    assert R.views_of([(0, 0), (0, 1), (1, 0)]) == 0


def test_vq_decode_arguments_are_checked_on_host():
    import ctypes
    from paper_2504_13339_amd import _lib
    lib = _lib.load()
    fake = ctypes.c_void_p(0x10000)
    f = (_lib.veg_vq_field * 2)(_lib.veg_vq_field(fake, 3), _lib.veg_vq_field(fake, 3))
    assert lib.veg_vq_decode(fake, 10, fake, 16, 7, f, 2, None) == 1          # widths 6 != dim 7
    assert b"sum" in lib.veg_last_error()
    assert lib.veg_vq_decode(fake, 10, fake, 0, 6, f, 2, None) == 1           # empty codebook
    assert lib.veg_vq_decode(fake, 10, fake, 16, 6, f, 9, None) == 1          # too many fields
    assert lib.veg_vq_decode(None, 0, None, 16, 6, f, 2, None) == 0           # nothing to decode


def test_densify_arguments_are_checked_on_host():
    import ctypes
    from paper_2504_13339_amd import _lib
    lib = _lib.load()
    fake = ctypes.c_void_p(0x10000)
    assert lib.veg_densify_workspace_bytes(1000) == (3 * 4 + 4) * 4
    f = (_lib.veg_densify_field * 1)(_lib.veg_densify_field(fake, fake, 4, 1))      # means must have width 3
    assert lib.veg_densify_apply(10, fake, fake, fake, fake, f, 1, fake, 1 << 20, None) == 1
    assert b"width 3" in lib.veg_last_error()
    f[0].width, f[0].role = 3, 7
    assert lib.veg_densify_apply(10, fake, fake, fake, fake, f, 1, fake, 1 << 20, None) == 1
    assert lib.veg_densify_plan(10, fake, fake, fake, None, ctypes.c_float(float("nan")), ctypes.c_float(0.0),
                                ctypes.c_float(0.0), fake, None, fake, 1 << 20, None) == 1
    assert lib.veg_densify_plan(10, fake, fake, fake, None, ctypes.c_float(0.1), ctypes.c_float(0.0),
                                ctypes.c_float(0.0), fake, None, fake, 4, None) == 1          # small workspace


def test_fused_projection_backward_arguments_are_checked_on_host():
    import ctypes
    from paper_2504_13339_amd import _lib
    lib = _lib.load()
    fake = ctypes.c_void_p(0x10000)
    # the densification outputs come as a pair: one without the other is refused first
    assert lib.veg_project_bwd_fused(None, None, None, fake, None, fake, None, 1, None) == 1
    assert b"both" in lib.veg_last_error()
    assert lib.veg_project_bwd_fused(None, None, None, fake, None, None, fake, 0, None) == 1


def test_shared_runs_must_share_a_camera():
    import pytest
    from paper_2504_13339_amd import render as R
    with pytest.raises(ValueError):
        R.train_step(None, None, None, [(0, 0), (1, 0)], None, None, 2, shared=2)
    with pytest.raises(ValueError):
        R.train_step(None, None, None, [(0, 0), (0, 1), (0, 2)], None, None, 2, shared=2)
    with pytest.raises(ValueError):
        R.train_step(None, None, None, [(0, 0), (0, 1), (1, 1), (1, 0)], None, None, 4, shared=True)


def test_backward_rejects_options_that_break_transmittance_recovery():
    """veg_render_bwd recovers T as T / (1 - alpha): alpha_clamp = 1 and t_min = 0 are
    rejected before any launch (the pointers are never dereferenced); the defaults pass
    the option check and fail later only on the fake hit-bit buffer."""
    import ctypes
    from paper_2504_13339_amd import _lib
    lib = _lib.load()
    fake = ctypes.c_void_p(0x10000)
    img = ctypes.c_void_p(0x20000)
    p = _lib.veg_proj(1, 1, 16, 16, 1, 1, 1, fake, fake, fake, fake)
    b = _lib.veg_bins(fake, fake, fake, fake, fake, 64, None, 0)
    for clamp, tmin in ((1.0, 1e-4), (0.99, 0.0), (0.9999, 1e-4)):
        o = _lib.veg_opts()
        lib.veg_opts_default(ctypes.byref(o))
        o.alpha_clamp, o.t_min = clamp, tmin
        assert lib.veg_render_bwd(ctypes.byref(p), ctypes.byref(b), ctypes.byref(o), img, img, img, img, None) == 1
        assert b"alpha_clamp" in lib.veg_last_error()
    o = _lib.veg_opts()
    lib.veg_opts_default(ctypes.byref(o))
    o.alpha_clamp, o.t_min = 0.999, 1e-20
    b.hits, b.hit_words = fake, 1
    assert lib.veg_render_bwd(ctypes.byref(p), ctypes.byref(b), ctypes.byref(o), img, img, img, img, None) == 1
    assert b"hit_words" in lib.veg_last_error()


# Declarations with no paper passage behind them: error reporting and the library version.
PLUMBING = {"veg_status_str": "error strings", "veg_last_error": "error message", "veg_version": "library version"}


def declaration_comments():
    """For every declared function: its own doc comment (the comment before it, shared by
    consecutive declarations) and the comment of the section divider it sits under."""
    text = open(HEADER).read()
    out = {}
    own, divider = "", ""
    pos = 0
    for m in re.finditer(r"/\*(.*?)\*/|\b(veg_[a-z0-9_]+)\s*\(", text, flags=re.S):
        if m.group(1) is not None:
            body = re.sub(r"\s*\n\s*\*\s?", " ", m.group(1))
            if body.lstrip().startswith("---"):
                divider, own = body, ""
            elif text[m.start() - 2:m.start()].strip() == "" or text[m.start() - 1] == "\n":
                # a doc comment on its own lines (not a trailing field comment)
                line_start = text.rfind("\n", 0, m.start()) + 1
                if text[line_start:m.start()].strip() == "":
                    own = body
        else:
            name = m.group(2)
            line_start = text.rfind("\n", 0, m.start()) + 1
            line = text[line_start:m.start()]
            if "(" in line or "*" in line.replace("*", "", 0) and "/*" in line:
                continue
            if name not in out:
                out[name] = (own, divider)
    return out


CITATION = re.compile(r'section "[^"]+"|Eq\. ?\d')


# The allocation-free variant names the callers it is for instead of a passage.
NO_ALLOC = {"veg_bin_static"}


def test_every_declaration_cites_the_passage_it_implements():
    """Each function of the boundary carries a citation of the paper's section or equation
    it implements, in its own comment or its section divider (plumbing excepted; the
    allocation-free variant names its callers: those that cannot allocate)."""
    comments = declaration_comments()
    assert set(declared_functions()) <= set(comments), set(declared_functions()) - set(comments)
    missing = [n for n in declared_functions() if n not in PLUMBING and n not in NO_ALLOC and
               not any(CITATION.search(c) for c in comments[n])]
    assert not missing, missing
    for n in NO_ALLOC:
        assert "cannot allocate" in comments[n][0], n


def test_bin_static_rejects_sizes_beyond_its_scratch_on_host():
    """veg_bin_static checks its arguments and its pair limit before touching the device
    (the pointers are never dereferenced)."""
    import ctypes
    from paper_2504_13339_amd import _lib
    lib = _lib.load()
    fake = ctypes.c_void_p(0x10000)
    status = ctypes.c_void_p(0x20000)
    b = _lib.veg_bins(fake, fake, fake, fake, fake, 64, None, 0)
    big = _lib.veg_proj(262145, 1, 16, 16, 1, 1, 1, fake, fake, fake, fake)
    assert lib.veg_bin_static(ctypes.byref(big), ctypes.byref(b), status, None) == 1
    assert b"262144" in lib.veg_last_error()
    two = _lib.veg_proj(131073, 2, 16, 16, 1, 1, 2, fake, fake, fake, fake)
    assert lib.veg_bin_static(ctypes.byref(two), ctypes.byref(b), status, None) == 1
    ok = _lib.veg_proj(1000, 1, 16, 16, 1, 1, 1, fake, fake, fake, fake)
    assert lib.veg_bin_static(ctypes.byref(ok), ctypes.byref(b), None, None) == 1
    assert b"status" in lib.veg_last_error()
    assert lib.veg_bin_static(ctypes.byref(ok), ctypes.byref(b), ctypes.c_void_p(0x20004), None) == 1
    assert lib.veg_bin_static(ctypes.byref(ok), None, status, None) == 1
