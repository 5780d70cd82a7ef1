"""Host-side checks of the C-ABI library that need no GPU: it builds, loads,
exports every symbol the header declares, and rejects invalid configurations
before touching a device."""
import os
import re

import pytest

from paper_2412_10167_amd import EXPORTED_SYMBOLS, load_library
from paper_2412_10167_amd.tdwp import Plan, TdwpError
from workloads import config

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    text = open(os.path.join(ROOT, "include", "tdwp.h")).read()
    return set(re.findall(r"^(?:int|void|const char\*)\s+(tdwp_\w+)\s*\(", text, re.M))


def test_header_and_binding_agree():
    assert header_symbols() == set(EXPORTED_SYMBOLS)


def test_option_and_statistic_codes_agree_with_the_header():
    from paper_2412_10167_amd.tdwp import OPTIONS, STATS
    text = open(os.path.join(ROOT, "include", "tdwp.h")).read()
    for prefix, table in (("TDWP_OPT_", OPTIONS), ("TDWP_STAT_", STATS)):
        declared = {m.group(1).lower(): int(m.group(2))
                    for m in re.finditer(prefix + r"(\w+)\s*=\s*(\d+)", text)}
        assert declared == table, prefix


def test_library_exports_every_declared_symbol():
    lib = load_library()
    for name in header_symbols():
        assert hasattr(lib, name), name


def test_strerror_codes():
    lib = load_library()
    assert lib.tdwp_strerror(0) == b"ok"
    assert b"invalid" in lib.tdwp_strerror(-1)
    assert b"order" in lib.tdwp_strerror(-4)


@pytest.mark.parametrize("field,value", [
    ("n_r", 1), ("n_gamma", 1), ("r_min", -1.0), ("n_elec", 0), ("n_elec", 9),
    ("r_flux", 100.0), ("R_inf", 0.1), ("n_energy", 1), ("ecol_max", 0.0),
])
def test_invalid_config_is_einval_without_a_device(field, value):
    s = config(1)
    s[field] = value
    with pytest.raises(TdwpError) as e:
        Plan(s, stream=None)
    assert e.value.code == -1


def test_invalid_units_are_einval():
    for unit in (dict(J=2, parity=1, omega_max=3, n_packets=1),     # omega_max > J
                 dict(J=2, parity=0, omega_max=0, n_packets=1),     # parity not +-1
                 dict(J=2, parity=-1, omega_max=0, n_packets=1),    # omega_min = 1 > omega_max
                 dict(J=3, parity=1, omega_max=2, n_packets=0)):    # no packets
        s = config(1)
        s["units"] = [unit]
        with pytest.raises(TdwpError) as e:
            Plan(s, stream=None)
        assert e.value.code == -1


def test_unimplemented_precision_is_rejected():
    s = config(1)
    with pytest.raises(KeyError):
        Plan(s, precision="fp8", stream=None)
