"""The GPU tests run the in-tree HIP library: the process has mapped
paper_2405_04690_amd/libgbl.so itself (there is no CPU fallback and no way to
point the binding at another build)."""
import os

import pytest

from paper_2405_04690_amd import build, gbl

pytestmark = pytest.mark.gpu


def test_in_tree_library_is_the_one_loaded():
    gbl.load_library()
    maps = open("/proc/self/maps").read()
    assert os.path.realpath(build.LIB_PATH) in maps
    mapped = {line.split()[-1] for line in maps.splitlines() if line.endswith("libgbl.so")}
    assert mapped == {os.path.realpath(build.LIB_PATH)}
