"""CODATA 2018 conversion factors; everything downstream works in atomic units."""
EH_EV = 27.211386245988          # 1 hartree in eV
AMU_ME = 1822.888486209          # 1 unified atomic mass unit in electron masses
ANG_BOHR = 1.0 / 0.529177210903  # 1 angstrom in bohr


def ev(x):
    """eV -> hartree."""
    return x / EH_EV


def amu(x):
    """amu -> electron masses."""
    return x * AMU_ME
