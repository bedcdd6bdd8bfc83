"""Host-side argument checks of the map bookkeeping binding: wrong dtypes, shapes and
devices are rejected before anything reaches the library (no GPU needed)."""

import pytest
import torch

from paper_2506_00970_amd import mapstate


def test_rejects_wrong_dtypes_and_shapes():
    f = torch.zeros(8)
    i = torch.zeros(8, dtype=torch.int32)
    with pytest.raises(TypeError):
        mapstate.covisibility_counts(f, i)
    with pytest.raises(ValueError):
        mapstate.covisibility_counts(f, torch.zeros(7))
    with pytest.raises(TypeError):
        mapstate.keyframe_test(torch.zeros(2), torch.zeros(12), torch.zeros(12))
    with pytest.raises(ValueError):
        mapstate.keyframe_test(torch.zeros(3, dtype=torch.int32), torch.zeros(12), torch.zeros(12))
    with pytest.raises(TypeError):
        mapstate.prune_mask(f, torch.zeros(8, dtype=torch.int64), 0)
    with pytest.raises(ValueError):
        mapstate.compact(torch.zeros((3, 8), dtype=torch.float64), None)
    with pytest.raises(TypeError):
        mapstate.compact(torch.zeros((3, 8)), torch.zeros(8, dtype=torch.bool))
    with pytest.raises(TypeError):
        mapstate.correct(torch.zeros((15, 8)), i.to(torch.int64), torch.zeros(2, 12))
    with pytest.raises(ValueError):
        mapstate.correct(torch.zeros((15, 8)), i, torch.zeros(2, 11))
    st = mapstate.MapState(8, "cpu")
    with pytest.raises(ValueError):
        st.update(torch.zeros((15, 8)), torch.zeros(9), torch.zeros(12), 1, inactive_after=5)
    st.active = st.active.to(torch.int64)
    with pytest.raises(TypeError):
        st.update(torch.zeros((15, 8)), torch.zeros(8), torch.zeros(12), 1, inactive_after=5)
