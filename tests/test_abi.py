"""Host-side checks of the C ABI that need no GPU.

* the built library loads and exports every function include/ecc.h declares;
* the Python binding's struct mirrors the C layout;
* the product package does not reach the oracle.
"""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ecc.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ecc_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for n in ("ecc_create", "ecc_compute", "ecc_compute_ex", "ecc_compute_batch", "ecc_destroy",
              "ecc_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2203_09087_amd import ecc
    if not os.path.exists(ecc.LIB_PATH):
        pytest.skip("libecc_hip.so not built")
    lib = ecc.load_library()
    for name in _declared_functions():
        assert hasattr(lib, name), name
    assert set(ecc.EXPORTED) == set(_declared_functions())
    out = subprocess.run(["nm", "-D", "--defined-only", ecc.LIB_PATH], capture_output=True, text=True)
    if out.returncode == 0:
        syms = set(re.findall(r"\s[TW]\s+(\S+)", out.stdout))
        for name in _declared_functions():
            assert name in syms, name


def test_descriptor_layout():
    from paper_2203_09087_amd import ecc
    im = ecc.ecc_image
    assert ctypes.sizeof(im) == 112 and ecc.ECC_MAX_NDIM == 8
    assert im.data.offset == 0 and im.ndim.offset == 8 and im.dtype.offset == 12
    assert im.dims.offset == 16 and im.range_mode.offset == 80 and im.reserved.offset == 84
    assert im.lo.offset == 88 and im.hi.offset == 96 and im.out.offset == 104
    with open(HEADER) as fh:
        assert re.search(r"#define ECC_MAX_NDIM (\d+)", fh.read()).group(1) == str(ecc.ECC_MAX_NDIM)


def test_create_without_device_reports_error():
    """On a machine without a GPU, ecc_create fails with a status and a message."""
    import torch
    from paper_2203_09087_amd import ecc
    if not os.path.exists(ecc.LIB_PATH):
        pytest.skip("libecc_hip.so not built")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(ecc.EccError) as ei:
        ecc.ecc_create(0, ecc.ECC_VERTEX)
    assert ei.value.status == ecc.ECC_ERR_DEVICE
    assert "device" in ecc.ecc_last_error(None)


def test_product_package_does_not_use_the_oracle():
    pkg = os.path.join(ROOT, "paper_2203_09087_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "ecc_oracle" not in text, f


def test_batch_descriptor_array_matches_structures():
    """make_images() writes the same bytes as one ecc_image structure per image
    (the batch calls pass its buffer as the ecc_image array)."""
    torch = pytest.importorskip("torch")
    from paper_2203_09087_amd import ecc
    imgs = [torch.zeros((5, 7), dtype=torch.uint8), torch.zeros((2, 3, 4), dtype=torch.int16),
            torch.zeros((3, 1, 2, 9), dtype=torch.float32), torch.zeros((1, 1), dtype=torch.float32)]
    outs = [torch.zeros(16, dtype=torch.int64) for _ in imgs]
    ranges = [None, "auto", (-1.5, 2.25), (0.0, float("inf"))]
    arr = ecc.make_images(imgs, outs, ranges)
    structs = (ecc.ecc_image * len(imgs))(*[ecc.make_image(t, o, r) for t, o, r in zip(imgs, outs, ranges)])
    assert arr.tobytes() == bytes(structs)
    assert len(ecc.make_images([], [])) == 0
    with pytest.raises(ValueError):
        ecc.make_images(imgs[:1], outs[:1], ["nearest"])
    with pytest.raises(ValueError):
        ecc.make_images([torch.zeros((4, 6), dtype=torch.uint8)[:, ::2]], outs[:1])
