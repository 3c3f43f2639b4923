"""The smoke check itself (one small forward + backward against the oracle),
run inside the GPU suite so that a mistake in the check surfaces here."""
import os
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_smoke_entry_point(capsys):
    from _helpers import device
    device()
    if ROOT not in sys.path:
        sys.path.insert(0, ROOT)
    import __graft_entry__ as g
    g.smoke()
    out = capsys.readouterr().out
    assert "smoke ok" in out and "grad rel err" in out
