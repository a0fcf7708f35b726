"""Host-side checks of the C ABI (no GPU needed): symbols and argument validation."""

import ctypes
import os
import re

import pytest
import torch

import paper_2504_15350_amd as rp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(rpod_[a-z_0-9]+)\s*\(", text))
    return names


needs_lib = pytest.mark.skipif(not os.path.exists(rp.LIB_PATH), reason="librpod.so not built")


@needs_lib
def test_library_exports_every_declared_symbol():
    L = rp.lib()
    syms = _declared_symbols()
    assert {"rpod_compute", "rpod_plan_create", "rpod_workspace_size"} <= syms
    for s in sorted(syms):
        assert hasattr(L, s), s


@needs_lib
@pytest.mark.parametrize("kw,status", [
    (dict(m=0, n=10, r=1, p=0, q=0), 1),
    (dict(m=10, n=10, r=0, p=0, q=0), 1),
    (dict(m=10, n=10, r=2, p=-1, q=0), 1),
    (dict(m=10, n=10, r=2, p=1, q=-1), 1),
    (dict(m=10, n=10, r=8, p=3, q=0), 1),            # l > min(m, n)
    (dict(m=1000, n=1000, r=100, p=29, q=0), 5),      # l > 128
    (dict(m=100, n=100, r=4, p=2, q=1, ld=99), 1),     # ld < m
    (dict(m=100, n=100, r=4, p=2, q=1, block_cols=-1), 1),   # negative block length
    (dict(m=100, n=100, r=4, p=2, q=1, block_cols=30), 1),   # n not a multiple of the block length
    (dict(m=100, n=64, r=4, p=2, q=1, block_cols=1), 1),     # one-column blocks: S' = 0
    (dict(m=100, n=20, r=15, p=2, q=1, block_cols=5), 1),    # l = 17 > n - blocks = 16
    (dict(m=1000, n=650, r=4, p=2, q=1, block_cols=10), 5),  # 65 blocks
    (dict(m=1000, n=400, r=100, p=10, q=1, block_cols=20), 5),  # roundup(l) + roundup(blocks) > 128
    (dict(m=100, n=100, r=4, p=2, q=1, flags=2), 1),           # unknown flag
    (dict(m=100, n=100, r=4, p=2, q=1, flags=1, block_cols=10), 5),  # energy with centring
])
def test_workspace_size_rejects(kw, status):
    ld = kw.pop("ld", None)
    with pytest.raises(rp.RpodError) as e:
        rp.workspace_size(dtype=torch.float32, ld=ld, **kw)
    assert e.value.status == status
    assert rp.lib().rpod_last_error().decode() != "no error"


@needs_lib
def test_workspace_size_accepts_edges():
    a = rp.workspace_size(1000, 30, 20, 10, 0, torch.float64)      # l == n
    b = rp.workspace_size(262144, 5000, 50, 10, 2, torch.float32)
    c = rp.workspace_size(4096, 200, 100, 28, 1, torch.float32)     # l == 128
    assert 0 < a < b and c > 0
    assert b % 256 == 0
    # fluctuation centring: the indicator and block-sum columns and the small buffers
    bc = rp.workspace_size(262144, 5000, 50, 10, 2, torch.float32, block_cols=500)
    assert bc > b and bc - b < 40 * 2 ** 20
    assert rp.workspace_size(1000, 640, 50, 14, 1, torch.float32, block_cols=10) > 0   # 64 blocks, l = 64
    assert rp.workspace_size(1000, 300, 100, 12, 1, torch.bfloat16, block_cols=300) > 0  # one block, l = 112
    # energy: the partial sums of ||S||_F^2
    assert rp.workspace_size(262144, 5000, 50, 10, 2, torch.float32, flags=rp.DESC_ENERGY) > b


@needs_lib
@pytest.mark.parametrize("dt", [torch.float64, torch.float32, torch.bfloat16, torch.float16])
def test_every_storage_dtype_has_a_plan(dt):
    assert rp.workspace_size(1000, 100, 10, 5, 1, dt) > 0


@needs_lib
def test_unknown_dtype_code_rejected():
    L = rp.lib()
    d = rp.make_desc(100, 50, 5, 5, 1, torch.float32)
    d.dtype = 7
    out = ctypes.c_size_t(0)
    assert L.rpod_workspace_size(ctypes.byref(d), ctypes.byref(out)) == 1


@needs_lib
def test_plan_create_null_arguments():
    L = rp.lib()
    d = rp.make_desc(100, 50, 5, 5, 1, torch.float32)
    h = ctypes.c_void_p()
    assert L.rpod_plan_create(ctypes.byref(h), ctypes.byref(d), None, 1 << 20, None) == 1
    assert L.rpod_plan_create(ctypes.byref(h), ctypes.byref(d), ctypes.c_void_p(256 * 3 + 8), 1 << 30, None) == 1
    assert L.rpod_plan_create(ctypes.byref(h), ctypes.byref(d), ctypes.c_void_p(1 << 20), 16, None) == 3
    assert L.rpod_compute(None, None, 0, None, None, None) == 1
    assert L.rpod_status_query(None, None) == 1
    assert L.rpod_plan_destroy(None) == 1
    assert L.rpod_generate_omega(1, 0, 4, 0, None, 1, None) == 1
    assert L.rpod_sketch_bits(1, 10, 4, None, None) == 1


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(rp, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(rp, "_lib", None)
    with pytest.raises(RuntimeError, match="not built"):
        rp.lib()


@needs_lib
def test_batched_workspace_validation():
    f32, f64 = torch.float32, torch.float64
    a = rp.make_desc(3000, 300, 10, 10, 2, f32)
    b = rp.make_desc(5000, 260, 25, 10, 2, f32)
    # a batch of one is the single-matrix plan
    assert rp.workspace_size_batched([a]) == rp.workspace_size(3000, 300, 10, 10, 2, f32)
    two = rp.workspace_size_batched([a, b])
    assert two > rp.workspace_size(3000, 300, 10, 10, 2, f32) + rp.workspace_size(5000, 260, 25, 10, 2, f32) // 2
    with pytest.raises(rp.RpodError) as e:
        rp.workspace_size_batched([a, rp.make_desc(3000, 300, 10, 10, 2, f64)])  # mixed dtype
    assert e.value.status == 1
    with pytest.raises(rp.RpodError) as e:
        rp.workspace_size_batched([a, rp.make_desc(3000, 300, 10, 10, 1, f32)])  # mixed q
    assert e.value.status == 1
    with pytest.raises(rp.RpodError) as e:
        rp.workspace_size_batched([a, rp.make_desc(3000, 300, 100, 29, 2, f32)])  # l > 128 in one member
    assert e.value.status == 5
    L = rp.lib()
    out = ctypes.c_size_t(0)
    arr = (rp._Desc * 1)(a)
    assert L.rpod_workspace_size_batched(arr, 0, ctypes.byref(out)) == 1
    assert L.rpod_workspace_size_batched(None, 1, ctypes.byref(out)) == 1
    assert L.rpod_compute_batched(None, None, None, None, None, None) == 1
    assert L.rpod_status_query_batched(None, None) == 1


@needs_lib
def test_batched_workspace_of_the_64_matrix_workload_fits_hbm():
    """The 64-matrix uneven batch: workspace well under the 288 GB of one GPU."""
    import synth
    shapes = synth.batch_shapes(64, seed=4)
    descs = [rp.make_desc(m, n, r, 10, 2, torch.bfloat16) for (m, n, r, _a) in shapes]
    ws = rp.workspace_size_batched(descs)
    assert 0 < ws < 40e9


@needs_lib
def test_tuning_validation_and_workspace():
    f32 = torch.float32
    descs = [rp.make_desc(3000, 300, 10, 10, 2, f32), rp.make_desc(5000, 2600, 25, 10, 2, f32)]
    base = rp.workspace_size_batched(descs)
    assert rp.workspace_size_batched(descs, rp.Tuning()) == base      # all-zero knobs are the defaults
    small = rp.workspace_size_batched(descs, rp.Tuning(128, 64))
    large = rp.workspace_size_batched(descs, rp.Tuning(8192, 256))
    assert small <= base <= large                                      # more row splits, more slab memory
    for bad in (rp.Tuning(-1, 0), rp.Tuning(0, 257), rp.Tuning(0, -3)):
        with pytest.raises(rp.RpodError) as e:
            rp.workspace_size_batched(descs, bad)
        assert e.value.status == 1
    t = rp.Tuning(256, 64)
    t.reserved[2] = 1
    with pytest.raises(rp.RpodError):
        rp.workspace_size_batched(descs, t)
    arr = (rp._Desc * 2)(*descs)
    need = ctypes.c_size_t(0)
    assert rp.lib().rpod_autotune_workspace_size(arr, 2, ctypes.byref(need)) == 0
    assert need.value > large                                          # trial plans plus their outputs
    best = rp.Tuning()
    assert rp.lib().rpod_autotune(arr, 2, None, None, 0, None, 1, None, ctypes.byref(best), None) == 1
