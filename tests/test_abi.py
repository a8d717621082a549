"""CPU checks of the C ABI boundary: the library loads, exports every
function include/pmmm.h declares, and validates parameters on the host
(pmmm_workspace_bytes makes no GPU call)."""
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    from paper_1409_5981_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1409_5981_amd import build
        build.build()
    return _lib.load()


def _declared():
    with open(os.path.join(ROOT, "include", "pmmm.h")) as f:
        src = f.read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(pmmm_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol(lib):
    from paper_1409_5981_amd import _lib
    names = _declared()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(_lib.EXPORTS) == names


def test_parameter_validation_on_host(lib):
    from paper_1409_5981_amd._lib import make_params, workspace_bytes
    ok = make_params(16, 5, "periodic")
    assert workspace_bytes(ok, 32768) > 0
    assert workspace_bytes(make_params(16, 5, "periodic", cutoff=3), 10) == 0      # bad cutoff
    assert workspace_bytes(make_params(4, 3, "periodic", cutoff=2), 10) == 0       # n < 2c+1
    assert workspace_bytes(make_params(8, 11, "open"), 10) == 0                    # p > PMAX
    assert workspace_bytes(make_params(8, 10, "open"), 10) > 0                     # p = PMAX
    assert workspace_bytes(make_params(16, 9, "periodic"), 10) > 0
    assert workspace_bytes(make_params(64, 10, "open"), 10) > 0                    # streamed column kernel
    assert workspace_bytes(make_params(12, 3, "periodic"), 10) > 0                 # direct DFTs
    assert workspace_bytes(make_params(9, 5, "periodic", cutoff=2), 10) > 0        # odd edge
    assert workspace_bytes(make_params(65, 3, "periodic"), 10) == 0                # > 64, not 2^k
    assert workspace_bytes(make_params(128, 3, "open"), 10) == 0                   # nf > 128
    assert workspace_bytes(make_params(64, 3, "open", precision="f64"), 10) == 0   # nf > 64 (FP64)
    prm = make_params(8, 3, "open")
    prm.box[1] = 2.0                                                              # non-cubic cells
    assert workspace_bytes(prm, 10) == 0
    # open meshes of any nx x ny x nz cubic cells sit in a power-of-two cube
    assert workspace_bytes(make_params(12, 6, "open", shape=(12, 6, 9)), 10) > 0
    assert workspace_bytes(make_params(3, 2, "open", box=0.75, shape=(3, 4, 5)), 10) > 0
    assert workspace_bytes(make_params(33, 3, "open", shape=(33, 20, 17)), 10) > 0   # in 64^3
    assert workspace_bytes(make_params(65, 3, "open", shape=(65, 3, 3)), 10) == 0    # 128^3: nf > 128
    assert workspace_bytes(make_params(24, 3, "open", precision="f64"), 10) > 0     # in 32^3
    assert workspace_bytes(make_params(8, 3, "periodic", shape=(8, 8, 4)), 10) == 0 # periodic: cubic
    assert workspace_bytes(make_params(24, 3, "periodic"), 10) > 0                  # direct DFTs


def test_workspace_grows_with_particles(lib):
    from paper_1409_5981_amd._lib import make_params, workspace_bytes
    prm = make_params(32, 7, "periodic")
    # per particle: cell, slot, permutation, sorted cell and sorted slot (5 ints),
    # the sorted record and the sorted-order results (2 x 4 floats); plus one
    # int per near-field tile of 64 targets, and the radix-sort histograms:
    # 512 ints per tile, sized for the most tiles any count up to 2^20 uses
    # (2^20 - 1 particles in 1024 tiles of 1024), with one scan sum per 4096
    # and the dense-cell P2M items (16 bytes each: one per 512 particles plus
    # one per cell of more than 64, at most n / 65 of them, then one entry per
    # split cell, at most half the partial slots) and partial sums (2 n / 512
    # slots of P + 1 = 65 floats)
    hist = 512 * 1024 - 512
    sums = 512 * 1024 // 4096 - 1
    slots = 2 * (1 << 20) // 512
    items = (1 << 20) // 512 + (1 << 20) // 65 + slots // 2
    assert (workspace_bytes(prm, 1 << 20) - workspace_bytes(prm, 0)
            == (1 << 20) * 52 + 4 * (1 << 14) + 4 * (hist + sums) + 16 * items + 4 * 65 * slots)


def test_error_strings(lib):
    for code in range(6):
        assert lib.pmmm_error_string(code).startswith(b"PMMM_")


def test_one_hip_runtime_mapped():
    """Loading the library binds it to the HIP (and HSA) runtime torch already
    mapped: a fresh process holds exactly one of each after _lib.load()."""
    import subprocess
    import sys
    code = (
        "import re, sys; sys.path.insert(0, %r)\n"
        "from paper_1409_5981_amd import _lib\n"
        "_lib.load()\n"
        "maps = open('/proc/self/maps').read()\n"
        "hip = set(re.findall(r'\\S*libamdhip64\\S*', maps))\n"
        "hsa = set(re.findall(r'\\S*libhsa-runtime64\\S*', maps))\n"
        "print(len(hip), len(hsa), sorted(hip))\n" % ROOT)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    nhip, nhsa = (int(v) for v in r.stdout.split()[:2])
    assert nhip == 1 and nhsa == 1, r.stdout


def test_buffer_validation_before_any_call():
    """Wrong length, dtype, layout or device is rejected before the C call
    (a short output would let the kernels write past its end)."""
    import torch
    from paper_1409_5981_amd._lib import check_buffers
    f32 = torch.float32
    ok = torch.zeros(10, dtype=f32)
    with pytest.raises(ValueError, match="expected 10 elements"):
        check_buffers((ok, torch.zeros(9, dtype=f32)), f32, 10, what="out")
    with pytest.raises(ValueError, match="expected"):
        check_buffers((torch.zeros(10, 2, dtype=f32),), f32, 20, shape=(10, 3), what="out")
    with pytest.raises(ValueError, match="dtype"):
        check_buffers((torch.zeros(10, dtype=torch.float64),), f32, 10)
    with pytest.raises(ValueError, match="contiguous"):
        check_buffers((torch.zeros(20, dtype=f32)[::2],), f32, 10)
    with pytest.raises(ValueError, match="GPU"):
        check_buffers((ok,), f32, 10)
    with pytest.raises(ValueError, match="None"):
        check_buffers((None,), f32, 10)


def test_coefficient_storage_calls_validate_on_host(lib):
    """Record sizes agree with the oracle's bit layout (Sec. 5.3), and bad
    orders, sizes, flags and pointers are refused before any GPU call."""
    import ctypes
    from oracle.storage import cell_words
    for p in range(11):
        assert lib.pmmm_coef_record_words(p) == cell_words(p)
    assert lib.pmmm_coef_record_words(-1) == -1 and lib.pmmm_coef_record_words(11) == -1
    dummy = ctypes.c_void_p(16)
    EINVAL = 1
    assert lib.pmmm_coef_pack_f32(11, 4, dummy, dummy, dummy, 1, None) == EINVAL
    assert lib.pmmm_coef_pack_f32(3, -1, dummy, dummy, dummy, 1, None) == EINVAL
    assert lib.pmmm_coef_pack_f32(3, 4, dummy, dummy, dummy, 2, None) == EINVAL
    assert lib.pmmm_coef_pack_f32(3, 4, None, dummy, dummy, 1, None) == EINVAL
    assert lib.pmmm_coef_pack_f32(3, 4, dummy, dummy, None, 1, None) == EINVAL
    assert lib.pmmm_coef_unpack_f32(3, 4, None, dummy, dummy, None) == EINVAL
    assert lib.pmmm_coef_unpack_f32(-1, 4, dummy, dummy, dummy, None) == EINVAL
    assert lib.pmmm_coef_compose_f32(3, 4, dummy, None, dummy, None) == EINVAL
    assert lib.pmmm_coef_compose_f32(3, (1 << 31) + 1, dummy, dummy, dummy, None) == EINVAL
    assert lib.pmmm_coef_split_f32(12, 4, dummy, dummy, dummy, None) == EINVAL
    assert lib.pmmm_coef_split_f32(3, 4, dummy, None, dummy, None) == EINVAL
    assert lib.pmmm_coef_compose_f32(3, 0, None, None, None, None) == 0         # empty: nothing to do


def test_batch_refuses_non_power_of_two_periodic_systems(lib):
    """Batches run the radix-2 stage kernels only: a periodic system whose
    edge is not a power of two is refused on the host (no GPU call)."""
    import ctypes
    from paper_1409_5981_amd._lib import Params, make_params
    arr = (Params * 2)(make_params(16, 4, "periodic"), make_params(12, 4, "periodic"))
    out = ctypes.c_void_p()
    assert lib.pmmm_batch_create(2, arr, None, ctypes.byref(out)) == 5      # PMMM_EUNSUPPORTED
    assert b"power-of-two" in lib.pmmm_last_error()
