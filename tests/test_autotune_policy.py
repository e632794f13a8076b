"""Tile-side policy of the autotuner (host logic, no GPU)."""
from dataclasses import dataclass

from paper_2607_02954_amd.autotune import TilePolicy, grid_class


@dataclass
class FakeWorld:
    nx: int
    ny: int


def test_grid_classes_and_policy():
    assert grid_class(FakeWorld(128, 128)) == "cells2^14"
    assert grid_class(FakeWorld(160, 128)) == "cells2^14"
    assert grid_class(FakeWorld(512, 512)) == "cells2^18"
    pol = TilePolicy({"cells2^14": 16, "cells2^18": 64})
    assert pol.side_for(FakeWorld(128, 130)) == 16
    assert pol.side_for(FakeWorld(512, 512)) == 64
    assert pol.side_for(FakeWorld(256, 256)) == 32          # unmeasured class: default
    p = pol.params(FakeWorld(512, 512), transfer="sorted")
    assert (p.nx, p.ny, p.tile, p.transfer) == (512, 512, 64, "sorted")
