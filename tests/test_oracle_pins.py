"""The oracle against facts outside itself (CPU only); see oracle_pins.py."""
import pytest

from tests import oracle_pins

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


@pytest.mark.parametrize("check", oracle_pins.ALL, ids=lambda f: f.__name__)
def test_pin(check):
    check()
