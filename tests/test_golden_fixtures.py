"""CPU checks of the stored oracle fixtures: each still matches the input generator.

A fixture of oracle output is written by a committed script that calls only oracle/;
its recorded network digest must equal the digest of the network the generator builds
now, else the fixture is stale and the GPU parity test that reads it would compare
against the wrong network.
"""
import importlib.util
import os

import numpy as np

from tn_inputs import configs


def _load(name):
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", name + ".py")
    spec = importlib.util.spec_from_file_location(name, path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


fx = _load("make_rqc30d12_amplitudes")


def test_rqc30d12_fixture_matches_generator():
    digest, amps = fx.read_fixture()
    _, net, best = configs.build(fx.NAME)
    assert digest == fx.network_digest(net, best)
    assert amps.shape == (2 ** len(net.open_labels),) == (512,)
    assert np.all(np.isfinite(amps)) and np.count_nonzero(amps) == amps.size
    # Porter-Thomas scale: |a|^2 averages 2^-30 over bitstrings; these 512 share their
    # closed bits, so only the order of magnitude is fixed
    mean_p = float(np.mean(np.abs(amps) ** 2))
    assert 2.0 ** -36 < mean_p < 2.0 ** -24
