"""The thresholds the paper states (tests/golden/paper_constants.txt) are the
ones the oracle and the bindings use by default."""
import inspect
import os

from oracle.freq64 import TAU_F
from oracle.insert64 import TAU_A

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    vals = {}
    with open(os.path.join(HERE, "golden", "paper_constants.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                name, value = line.split()[:2]
                vals[name] = float(value)
    return vals


def test_oracle_uses_the_papers_thresholds():
    g = _golden()
    assert TAU_A == g["tau_a"] and TAU_F == g["tau_f"]


def test_binding_defaults_use_the_papers_thresholds():
    from paper_2512_08498_amd import frequency, rasterizer

    g = _golden()
    assert frequency.TAU_F == g["tau_f"]
    assert inspect.signature(frequency.Frequency.schedule).parameters["tau_f"].default == g["tau_f"]
    assert inspect.signature(rasterizer.Rasterizer.log_insert).parameters["tau_a"].default == g["tau_a"]
