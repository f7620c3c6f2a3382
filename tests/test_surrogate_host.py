"""Host logic of the surrogate pipeline (no GPU)."""
from paper_2606_16765_amd import surrogate


def test_field_model_parameter_range():
    fm = surrogate.FieldModel(surrogate.Config(), None, None, None)
    assert fm.in_range(1000.0, 0.0) and fm.in_range(10000.0, 15.0) and fm.in_range(5500.0, -15.0)
    assert not fm.in_range(999.0, 0.0) and not fm.in_range(10001.0, 0.0)
    assert not fm.in_range(5000.0, 15.5) and not fm.in_range(5000.0, -20.0)
    narrow = surrogate.FieldModel(surrogate.Config(), None, None, None, re_range=(2000.0, 3000.0), aoa_max=5.0)
    assert narrow.in_range(2500.0, 5.0) and not narrow.in_range(3500.0, 0.0) and not narrow.in_range(2500.0, 6.0)


def test_inner_mask_box():
    m = surrogate.inner_mask(128, 64, 64)
    assert m.sum() == (int(0.9 * 128) - int(0.1 * 128)) * 32 * 32
    assert m[12, 16, 16] == 1 and m[11, 16, 16] == 0 and m[12, 15, 16] == 0 and m[115, 47, 47] == 0
