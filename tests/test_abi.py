"""Host-side checks of the C-ABI library (no GPU needed): it loads, exports
every function include/ibl.h declares, and validates descriptors."""
import ctypes
import os
import re

import pytest

from paper_1704_04551_amd import ibl

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "ibl.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ibl_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = ibl.lib()
    names = declared_functions()
    assert len(names) >= 19
    for n in names:
        assert hasattr(L, n), n


def test_library_links_hip_runtime_only():
    """The product library is the HIP build: it depends on the HIP runtime and
    on nothing from the oracle."""
    import subprocess
    out = subprocess.run(["readelf", "-d", ibl.LIB_PATH], capture_output=True, text=True).stdout
    assert "libamdhip64" in out
    assert "oracle" not in out


def _desc(**kw):
    base = dict(n=(32, 32, 32), tau=1.0, storage="f32")
    base.update(kw)
    return ibl.make_desc(**base)


def test_brick_width_changes_layout_not_validity():
    """Every allowed brick width is a valid description; narrower bricks mean
    more candidate lists (the arena grows)."""
    kw = dict(n=(64, 36, 20), max_nodes=1000, max_meshes=1, max_templates=1, max_template_nodes=1000,
              max_template_edges=3000)
    sizes = [ibl.sim_bytes(_desc(brick_x=bx, **kw)) for bx in (64, 32, 16)]
    assert sizes[0] == ibl.sim_bytes(_desc(brick_x=0, **kw))  # 64 is the default for nx = 64
    assert sizes[0] <= sizes[1] <= sizes[2]


def test_sim_bytes_scales_with_storage():
    b64 = ibl.sim_bytes(_desc(storage="f64"))
    b32 = ibl.sim_bytes(_desc(storage="f32"))
    b16 = ibl.sim_bytes(_desc(storage="f16"))
    nc = 32 ** 3
    # two A/B copies of 19 populations dominate
    assert b64 - b32 >= 2 * 19 * nc * 4
    assert b32 - b16 >= 2 * 19 * nc * 2
    assert b16 >= 2 * 19 * nc * 2


@pytest.mark.parametrize("kw", [dict(tau=0.5), dict(tau=0.3), dict(n=(3, 32, 32)), dict(storage=7),
                                dict(delta=5), dict(init_profile=3), dict(max_nodes=-1),
                                dict(brick_x=8), dict(brick_x=128), dict(skin=2), dict(skin=-1),
                                dict(n=(32768, 4, 4)),
                                dict(n=(1024, 1024, 1024), storage="f32")])
def test_invalid_descriptor_rejected(kw):
    with pytest.raises(ibl.IBLError) as e:
        ibl.sim_bytes(_desc(**kw))
    assert e.value.status == -1


def test_null_arguments_rejected():
    L = ibl.lib()
    out = ctypes.c_size_t()
    assert L.ibl_sim_bytes(None, ctypes.byref(out)) == -1
    assert L.ibl_step(None, 1) == -1
    assert L.ibl_sync(None) == -1
    assert L.ibl_batch_create(None, 0, None) == -1
    assert L.ibl_last_error()
