"""The entry point's smoke check (one small thick-restart solve on the GPU
against the oracle) runs as a GPU test too."""
import pytest


@pytest.mark.gpu
def test_graft_entry_smoke():
    import __graft_entry__
    __graft_entry__.smoke()
