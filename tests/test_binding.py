"""Host-side checks of the Python binding that need neither a GPU nor the built
library: the binding refuses tensors whose memory does not hold their values, and
the autograd wrapper resolves such views before handing memory to the library."""

import pytest

from paper_1501_04950_amd import dwa

torch = pytest.importorskip("torch")


def _field():
    g = torch.Generator().manual_seed(5)
    return torch.complex(torch.randn(6, 4, 3, generator=g, dtype=torch.float64),
                         torch.randn(6, 4, 3, generator=g, dtype=torch.float64))


def test_lazy_conjugate_and_negative_views_are_refused():
    x = _field()
    dwa.check_storage(x)
    assert x.conj().is_conj() and x.conj().is_contiguous()
    with pytest.raises(ValueError):
        dwa.check_storage(x.conj())
    with pytest.raises(ValueError):
        dwa.check_storage(torch._neg_view(x))
    dwa.check_storage(x.conj().resolve_conj())


def test_autograd_inputs_are_resolved_to_their_values():
    from paper_1501_04950_amd import autograd as dag
    x = _field()
    for v in (x.conj(), torch._neg_view(x), x.conj().conj()):
        p = dag._plain(v)
        assert not p.is_conj() and not p.is_neg() and p.is_contiguous()
        # the memory now holds the view's values
        assert torch.equal(torch.view_as_real(p), torch.view_as_real(v.resolve_conj().resolve_neg()))
    # a lazy conjugate really does keep the other numbers in memory
    c = x.conj()
    assert torch.equal(torch.view_as_real(c.resolve_conj()), torch.view_as_real(torch.conj_physical(x)))
    assert c.data_ptr() == x.data_ptr()
