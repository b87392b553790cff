"""C-ABI checks that need no GPU: the library loads, exports every entry point the
header declares, and its host-side geometry agrees with the oracle's independent one."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import ntc_oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _header_functions():
    src = open(os.path.join(ROOT, "include", "ntc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ntc_[a-z0-9_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def ntc():
    from paper_2305_17105_amd import ntc as mod
    return mod


def test_every_declared_symbol_is_exported(ntc):
    import ctypes
    lib = ctypes.CDLL(ntc.LIB_PATH)
    names = _header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(ntc.exported_symbols())


@pytest.mark.parametrize("args", [
    (1024, 1024, 9, 8, 8, 4, 4, 64, 0, 2),
    (2048, 2048, 12, 12, 12, 4, 4, 64, 0, 2),
    (4096, 4096, 16, 16, 16, 2, 4, 64, 0, 2),
    (256, 256, 8, 8, 8, 4, 4, 64, 1, 2),
    (512, 128, 3, 5, 7, 2, 8, 32, 0, 1),
    (4096, 4096, 9, 12, 10, 2, 4, 64, 0, 1),
])
def test_host_geometry_matches_oracle(ntc, args):
    W, H, C, c0, c1, b0, b1, hd, M, sh = args
    m = ntc.material_init(W, H, C, c0, c1, b0, b1, hd, num_mips=M, grid_shift=sh)
    g = O.make_geometry(W, H, C, c0, c1, b0, b1, Hd=hd, M=M or None, shift=sh)
    assert m.num_mips == g.M and m.num_levels == g.J and m.input_width == g.K
    assert list(m.level_of_mip)[:g.M] == g.level_of_mip
    assert list(m.mip_w)[:g.M] == g.mip_w and list(m.mip_h)[:g.M] == g.mip_h
    for j in range(g.J):
        assert (m.g0_w[j], m.g0_h[j]) == g.g0[j] and (m.g1_w[j], m.g1_h[j]) == g.g1[j]
        assert m.g0_offset[j] == g.g0_off[j] and m.g1_offset[j] == g.g1_off[j]
    assert m.latent_count == g.latent_count
    assert list(m.mip_offset)[:g.M] == g.mip_off and m.target_count == g.target_count
    assert m.mlp_params == O.mlp_param_count(g.K, hd, C)
    # packed size: the oracle packer's output length (each grid padded to 16 bytes)
    assert m.packed_bytes == len(O.quantize_latents(g, np.zeros(g.latent_count)))


@pytest.mark.parametrize("bad", [
    dict(width=100), dict(channels=0), dict(channels=17), dict(c0=0), dict(b0=3), dict(hidden=40),
    dict(num_mips=20), dict(grid_shift=12), dict(width=4, height=4, grid_shift=2), dict(activation=5),
])
def test_invalid_descriptors_rejected(ntc, bad):
    kw = dict(width=256, height=256, channels=8, c0=8, c1=8, b0=4, b1=4, hidden=64, num_mips=0, grid_shift=2,
              activation=0)
    kw.update(bad)
    with pytest.raises(ntc.NtcError) as e:
        ntc.material_init(kw["width"], kw["height"], kw["channels"], kw["c0"], kw["c1"], kw["b0"], kw["b1"],
                          kw["hidden"], kw["num_mips"], kw["grid_shift"], kw["activation"])
    assert e.value.status == ntc.E_INVALID


def test_modified_descriptor_rejected_before_any_launch(ntc):
    import ctypes
    m = ntc.material_init(256, 256, 8, 8, 8, 4, 4, 64)
    m.latent_count += 1
    lib = ctypes.CDLL(ntc.LIB_PATH)
    lib.ntc_quantize_latents.restype = ctypes.c_int
    st = lib.ntc_quantize_latents(ctypes.byref(m), ctypes.c_void_p(16), ctypes.c_void_p(16), None)
    assert st == ntc.E_INVALID


def test_supported_shapes_and_sizes(ntc):
    m = ntc.material_init(2048, 2048, 12, 12, 12, 4, 4, 64)
    assert ntc.shape_supported(m, True) and ntc.shape_supported(m, False)
    m2 = ntc.material_init(256, 256, 3, 5, 7, 4, 4, 64)
    assert not ntc.shape_supported(m2, True)
    # FP16 packs are half the FP32 ones (plus FP32 biases)
    assert ntc.train_packed_bytes(m, ntc.F16) * 2 >= ntc.train_packed_bytes(m, ntc.F32) - 16
    assert ntc.mlp_packed_bytes(m, ntc.F32) > ntc.mlp_packed_bytes(m, ntc.F16) > 0
    assert ntc.mlp_packed_bytes(m, 7) == 0
    # FP8: 12 channels x 4 bits is not whole words -> unsupported; 16 x 2-bit is
    assert ntc.mlp_packed_bytes(m, ntc.FP8_E4M3) == 0
    m3 = ntc.material_init(4096, 4096, 16, 16, 16, 2, 4, 64)
    # e4m3 weights (96 + 64 + 16 slots x 64 lanes, one byte each) + 16 B scales + FP32 biases
    assert ntc.mlp_packed_bytes(m3, ntc.FP8_E4M3) == 4 * 24 * 64 + 4 * 16 * 64 + 16 * 64 + 16 + (2 * 64 + 16) * 4
    assert ntc.mlp_packed_bytes(m3, ntc.F16) > ntc.mlp_packed_bytes(m3, ntc.FP8_E4M3)


def test_decode_tile_rejects_bad_rectangles(ntc):
    """Rectangle checks happen before any launch: no GPU needed."""
    m = ntc.material_init(512, 512, 16, 16, 16, 2, 4, 64)
    fake = ctypes.c_void_p(16)
    lib = ntc._lib
    def call(lod, x0, y0, w, h, out=fake):
        return lib.ntc_decode_tile(ctypes.byref(m), fake, fake, ntc.F16, lod, x0, y0, w, h, out, ntc.F16, None)
    assert call(-1, 0, 0, 1, 1) == ntc.E_INVALID
    assert call(int(m.num_mips), 0, 0, 1, 1) == ntc.E_INVALID
    assert call(1, 200, 0, 57, 1) == ntc.E_INVALID        # mip 1 is 256 wide
    assert call(0, 0, 0, -1, 1) == ntc.E_INVALID
    assert call(0, 0, 0, 0, 7) == ntc.OK                   # empty: no-op
    assert call(0, 0, 0, 4, 4, out=None) == ntc.E_INVALID  # NULL output
    assert lib.ntc_decode_tile(ctypes.byref(m), fake, fake, 9, 0, 0, 0, 1, 1, fake, ntc.F16, None) == \
        ntc.E_UNSUPPORTED


@pytest.mark.parametrize("W,C,hd", [(4096, 16, 64), (4096, 12, 64), (4096, 8, 32), (2048, 12, 64)])
def test_training_plans_fit_large_materials(ntc, W, C, hd):
    """Plans (tile sizes, bin counts, workspace) exist for 4096^2 materials in both precisions."""
    m = ntc.material_init(W, W, C, C, C, 4, 4, hd)
    for prec in (ntc.F32, ntc.F16):
        assert ntc.train_workspace_bytes(m, 262144, prec) > 0


def test_decode_table_sizes_and_validation():
    """The grouped-decode table: header plus one entry per material; set-up calls with
    missing buffers fail before touching a device."""
    import ctypes as C
    from paper_2305_17105_amd import ntc
    assert ntc._lib.ntc_decode_table_bytes(0) == 0
    one = ntc._lib.ntc_decode_table_bytes(1)
    assert one > 256 and ntc._lib.ntc_decode_table_bytes(3) - one == 2 * (one - 256)
    m = ntc.material_init(256, 256, 8, 8, 8, 4, 4, 64)
    mats = ntc._materials([m])
    null = (C.c_void_p * 1)(None)
    st = ntc._lib.ntc_decode_table_init(mats, 1, null, null, ntc.F16, None, one)
    assert st == ntc.E_INVALID
    off = (C.c_int64 * 2)(0, 0)
    st = ntc._lib.ntc_decode_grouped(mats, 1, None, ntc.F16, None, off, None, ntc.F16, None)
    assert st == ntc.E_INVALID


def test_train_table_validation():
    """Grouped-training set-up rejects missing arguments before touching a device."""
    import ctypes as C
    from paper_2305_17105_amd import ntc
    assert ntc._lib.ntc_train_table_bytes(0) == 0
    assert ntc._lib.ntc_train_table_bytes(2) > ntc._lib.ntc_train_table_bytes(1) > 256
    m = ntc.material_init(256, 256, 8, 8, 8, 4, 4, 64)
    off = (C.c_int64 * 2)(0, 100)
    tg = (C.c_void_p * 1)(None)
    st = ntc._lib.ntc_train_table_init(ntc._materials([m]), 1, None, off, tg, ntc.F16, None, 0, None, 0)
    assert st == ntc.E_INVALID
    hp = ntc.hparams(precision=ntc.F16)
    st = ntc._lib.ntc_train_step_grouped(ntc._materials([m]), 1, None, None, off, tg, C.byref(hp), None, 0, None,
                                         None)
    assert st == ntc.E_INVALID


def test_training_sample_count_limit(ntc):
    """Training binning uses 32-bit list positions (up to 4 entries per sample): n above
    (2^31 - 1) / 4 is rejected with NTC_E_UNSUPPORTED before anything touches a device,
    and the workspace query returns 0 for it."""
    import ctypes as C
    m = ntc.material_init(256, 256, 8, 8, 8, 4, 4, 64)
    limit = (2 ** 31 - 1) // 4
    assert ntc.train_workspace_bytes(m, limit + 1, ntc.F32) == 0
    assert ntc._lib.ntc_backward_workspace_bytes(C.byref(m), limit + 1, ntc.F16) == 0
    fake = C.c_void_p(4096)  # aligned, never dereferenced: validation fails first
    st = ntc.TrainStateC(*([fake] * len(ntc.TrainStateC._fields_)))
    for prec in (ntc.F32, ntc.F16):
        hp = ntc.hparams(precision=prec)
        for call in (ntc._lib.ntc_train_step, ntc._lib.ntc_train_gradients):
            r = call(C.byref(m), C.byref(st), fake, limit + 1, fake, C.byref(hp), fake, 2 ** 40, None)
            assert r == ntc.E_UNSUPPORTED
        r = ntc._lib.ntc_train_update(C.byref(m), C.byref(st), limit + 1, C.byref(hp), fake, 2 ** 40, None)
        assert r == ntc.E_UNSUPPORTED
        r = ntc._lib.ntc_backward(C.byref(m), fake, fake, fake, prec, fake, limit + 1, fake, 1.0, fake, fake, fake,
                                  2 ** 40, None)
        assert r == ntc.E_UNSUPPORTED
        assert "2^31" in ntc._lib.ntc_last_error().decode()


def test_noalloc_step_rejects_steps_beyond_its_scratch(ntc):
    """ntc_train_step_noalloc returns NTC_E_WORKSPACE, before anything touches a device,
    when the step's workspace exceeds the static scratch array (a 2^20-sample step on a
    2048^2 x 12 material), and validates like ntc_train_step."""
    import ctypes as C
    assert ntc.NOALLOC_SCRATCH_BYTES == 128 << 20
    m = ntc.material_init(2048, 2048, 12, 12, 12, 4, 4, 64)
    fake = C.c_void_p(4096)  # aligned, never dereferenced: validation fails first
    st = ntc.TrainStateC(*([fake] * len(ntc.TrainStateC._fields_)))
    for prec in (ntc.F32, ntc.F16):
        hp = ntc.hparams(precision=prec)
        r = ntc._lib.ntc_train_step_noalloc(C.byref(m), C.byref(st), fake, 2 ** 20, fake, C.byref(hp), None)
        assert r == ntc.E_WORKSPACE, r
        assert "static array" in ntc._lib.ntc_last_error().decode()
        r = ntc._lib.ntc_train_step_noalloc(C.byref(m), C.byref(st), None, 4096, fake, C.byref(hp), None)
        assert r == ntc.E_INVALID
        r = ntc._lib.ntc_train_step_noalloc(C.byref(m), C.byref(st), fake, 0, fake, C.byref(hp), None)
        assert r == ntc.E_INVALID


def test_table3_profiles_supported_with_table6_level0_bytes(ntc):
    """Table 3's four profiles on the table's 4096^2 x 9 reference set: decode and training
    kernels exist (with the paper's network: hardGELU, LOD input), and the library's
    packed level-0 grids take exactly the 4k column of Table 6 (tests/golden)."""
    import json
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "table6_storage.json")))
    for name, p in gold["profiles"].items():
        m = ntc.material_init(4096, 4096, 9, p["c0"], p["c1"], p["b0"], p["b1"], 64, grid_shift=p["shift"],
                              activation=ntc.ACT_HARDGELU, lod_input=1)
        assert ntc.shape_supported(m, True) and ntc.shape_supported(m, False), name
        level0 = (m.g0_packed[1] if m.num_levels > 1 else m.packed_bytes) - m.g0_packed[0]
        assert level0 == gold["grids_mb"][name]["4096"] * 2 ** 20, (name, level0)
        assert ntc.train_workspace_bytes(m, 262144, ntc.F16) > 0, name
        # FP32 training sums latent gradients in 8-byte fixed point: with G0 at 2048^2 (NTC
        # 2.25 at 4k) its 8 x 8 tiles outnumber the binning capacity; at 2k every profile fits
        m2 = ntc.material_init(2048, 2048, 9, p["c0"], p["c1"], p["b0"], p["b1"], 64, grid_shift=p["shift"],
                               activation=ntc.ACT_HARDGELU, lod_input=1)
        assert ntc.train_workspace_bytes(m2, 262144, ntc.F32) > 0, name
