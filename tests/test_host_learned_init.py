"""Host logic of the learned-initialisation workloads: where the training crops lie and which
part of the object the network's prediction initialises."""
import pytest

pytest.importorskip("torch")


def test_config3_trains_and_initialises_the_centre_crop():
    from paper_2205_03902_amd import configs, learned_init
    s = learned_init.setup_for(3)
    assert s.geo is configs.CFG3 and s.sweeps == 20 and s.geo.n_slices == 6
    o = (320 - 256) // 2
    assert s.train_offsets() == [(o, o)] and s.window == (o, o, 256, 256)


def test_config4_trains_on_tiles_and_initialises_the_whole_object():
    from paper_2205_03902_amd import configs, learned_init
    s = learned_init.setup_for(4)
    assert s.geo is configs.CFG4 and s.sweeps == 30 and s.geo.n_slices == 12
    tiles = s.train_offsets()
    assert len(tiles) == 16 and len(set(tiles)) == 16
    covered = {(y0 + dy, x0 + dx) for y0, x0 in tiles for dy in (0, 255) for dx in (0, 255)}
    assert min(covered) == (0, 0) and max(covered) == (1023, 1023)
    assert all(y0 % 256 == 0 and x0 % 256 == 0 for y0, x0 in tiles)
    assert s.window == (0, 0, 1024, 1024)


def test_tiles_must_cover_the_object():
    from paper_2205_03902_amd import configs, learned_init
    with pytest.raises(ValueError):
        learned_init.Setup(geo=configs.CFG4, grid=3).train_offsets()
    with pytest.raises(ValueError):
        learned_init.setup_for(2)
