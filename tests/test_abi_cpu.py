"""CPU checks of the C ABI: the library loads, exports every function the header
declares, its structures match the ctypes mirror, and argument validation runs
before any device work."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2307_11107_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "apic.h")


def _declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(apic_\w+)\s*\(", text, re.M)))


def test_header_declares_the_boundary():
    names = _declared_functions()
    for required in ("apic_init", "apic_inject", "apic_step", "apic_solve_poisson", "apic_tallies"):
        assert required in names
    assert set(names) == set(_abi.PROTOTYPES), "ctypes prototypes out of sync with the header"


def test_library_exports_every_declared_symbol():
    lib = _abi.load()
    for name in _declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", _abi.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (apic_\w+)", out))
    assert set(_declared_functions()) <= exported


def test_struct_layouts_match_header(tmp_path):
    src = tmp_path / "sz.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "apic.h"\n'
                   'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu\\n", sizeof(apic_species),'
                   ' sizeof(apic_grain_cfg), sizeof(apic_opts), sizeof(apic_tally),'
                   ' sizeof(apic_kernel_times), offsetof(apic_tally, count), offsetof(apic_opts, stream));'
                   'return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    want = [C.sizeof(_abi.apic_species), C.sizeof(_abi.apic_grain_cfg), C.sizeof(_abi.apic_opts),
            C.sizeof(_abi.apic_tally), C.sizeof(_abi.apic_kernel_times),
            _abi.apic_tally.count.offset, _abi.apic_opts.stream.offset]
    assert got == want


def _sp(**kw):
    import paper_2307_11107_amd as apic
    base = dict(q=-1, m=1, n_macro=10)
    base.update(kw)
    return apic.species(**base)


def _cfg(**kw):
    import paper_2307_11107_amd as apic
    base = dict(alpha=0.1, n1=16, n2=16, species_list=[apic.species(-1, 1, n_macro=10)])
    base.update(kw)
    return apic.grain_cfg(**base)


@pytest.mark.parametrize("kw,code", [(dict(alpha=0.25), _abi.APIC_ERANGE), (dict(alpha=-0.3), _abi.APIC_ERANGE),
                                     (dict(x1_out=0.0), _abi.APIC_ERANGE), (dict(x1_out=-1.0), _abi.APIC_ERANGE),
                                     (dict(n1=4), _abi.APIC_ERANGE), (dict(n2=4000), _abi.APIC_ERANGE),
                                     (dict(dt=0.0), _abi.APIC_EINVAL), (dict(kappa=-1.0), _abi.APIC_EINVAL),
                                     (dict(n1=2049), _abi.APIC_ERANGE), (dict(n2=2047), _abi.APIC_ERANGE),
                                     (dict(n_bins=-1), _abi.APIC_EINVAL),
                                     (dict(species_list=[]), _abi.APIC_EINVAL),
                                     (dict(species_list=[_sp(n_macro=2_000_000_001)]), _abi.APIC_ERANGE),
                                     (dict(species_list=[_sp(capacity=-1)]), _abi.APIC_EINVAL),
                                     (dict(species_list=[_sp(weight=-1.0)]), _abi.APIC_EINVAL),
                                     (dict(species_list=[_sp(T=-0.5)]), _abi.APIC_EINVAL),
                                     (dict(species_list=[_sp(m=0.0)]), _abi.APIC_EINVAL)])
def test_invalid_configurations_rejected_before_device_work(kw, code):
    import paper_2307_11107_amd as apic
    with pytest.raises(apic.ApicError) as e:
        apic.apic_init([_cfg(**kw)], apic.opts())
    assert e.value.code == code
    assert apic.apic_last_error(None)


def test_null_arguments():
    lib = _abi.load()
    assert lib.apic_init(None, 1, None, None) == _abi.APIC_EINVAL
    h = C.c_void_p()
    assert lib.apic_init(None, 1, None, C.byref(h)) == _abi.APIC_EINVAL
    assert lib.apic_step(None, 1) == _abi.APIC_EINVAL
    assert lib.apic_free(None) == _abi.APIC_OK
