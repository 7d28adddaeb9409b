"""CPU checks of the Python binding's argument marshalling (no GPU needed)."""
import types

import pytest

pytest.importorskip("torch")

from paper_2602_07853_amd import mpmlite


def test_every_option_reaches_the_struct():
    """Each field of the C options struct is filled from the option dict by
    name, so an option added to the struct cannot silently arrive as zero."""
    names = [f for f, _ in mpmlite._Opts._fields_]
    opts = mpmlite.default_opts()
    assert set(names) == set(opts), set(names) ^ set(opts)
    # distinct non-default values for every field
    probe = {}
    for i, name in enumerate(names):
        v = opts[name]
        probe[name] = (type(v)(i + 2) if isinstance(v, int) else float(i) + 0.25)
    c = mpmlite.Context._copts(types.SimpleNamespace(opts=probe))
    for name in names:
        assert getattr(c, name) == pytest.approx(probe[name]), name
