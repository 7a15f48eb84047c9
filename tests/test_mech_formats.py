"""The JSON front end and mechanism serialization (CPU, through the C ABI).

A mechanism written as JSON and read back by the library compiles to exactly the tables of
the same mechanism given as arrays (their packed bytes are equal); a packed mechanism
unpacks to identical tables and the same table program results; malformed inputs are
rejected with a message naming the problem.
"""
import json

import numpy as np
import pytest

from paper_2111_07436_amd import mechanism_json as MJ
from paper_2111_07436_amd import workloads as W

camp = pytest.importorskip("paper_2111_07436_amd.camp", reason="libcamp.so not built")


@pytest.mark.parametrize("name", ["c1", "c3", "zoo"])
def test_json_round_trip_compiles_identically(name):
    mech = W.make_mechanism(name)
    a = camp.Mech(mech)
    b = camp.Mech.from_json(MJ.to_json(mech, indent=1))
    assert a.info == b.info
    for x, y in zip(a.export(), b.export()):
        assert np.array_equal(x, y)
    assert a.pack() == b.pack()


def _expect(text, fragment):
    with pytest.raises(camp.CampError) as e:
        camp.Mech.from_json(text)
    assert e.value.code == camp.EINVAL
    assert fragment in str(e.value), str(e.value)


def test_json_errors_name_the_problem():
    ok = MJ.to_dict(W.make_mechanism("zoo"))
    _expect("{\"species\": [", "JSON")
    _expect("[1, 2]", "object")
    bad = json.loads(json.dumps(ok))
    bad["processes"][0]["reactants"] = {"NOPE": 1}
    _expect(json.dumps(bad), "NOPE")
    bad = json.loads(json.dumps(ok))
    bad["processes"][3]["type"] = "MAGIC"
    _expect(json.dumps(bad), "type")
    bad = json.loads(json.dumps(ok))
    del bad["processes"][6]["kinf"]
    _expect(json.dumps(bad), "TROE")
    bad = json.loads(json.dumps(ok))
    bad["species"][13]["phase"] = "nowhere"
    _expect(json.dumps(bad), "nowhere")
    bad = json.loads(json.dumps(ok))
    bad["processes"][0]["A"] = -1.0                       # camp_mech_load validation
    _expect(json.dumps(bad), "reaction 0")


def test_json_reactant_multiplicity_and_defaults():
    doc = {"species": [{"name": "HO2"}, {"name": "H2O2"}],
           "processes": [{"type": "ARRHENIUS", "reactants": {"HO2": 2}, "products": {"H2O2": 1.0},
                          "A": 1e-12}]}
    m = camp.Mech.from_json(json.dumps(doc))
    ref = camp.Mech(W.Mechanism([W.Species("HO2"), W.Species("H2O2")], [],
                                [W.Reaction(W.RXN_ARRHENIUS, [0, 0], [1], [1.0], [1e-12, 0, 0, 300, 0, 0])]))
    assert m.pack() == ref.pack()


@pytest.mark.parametrize("name", ["c2", "c5", "zoo"])
def test_pack_unpack_identical(name, rng):
    a = camp.Mech(W.make_mechanism(name))
    blob = a.pack()
    b = camp.Mech.unpack(blob)
    assert a.info == b.info and b.pack() == blob
    for x, y in zip(a.export(), b.export()):
        assert np.array_equal(x, y)
    for lanes in (64, 128, 256):
        if lanes > 64 and a.n_state <= lanes // 2:
            continue
        assert a.layout_info(lanes) == b.layout_info(lanes)
    # the table program gives the same bits
    perm, rp, col, p0 = a.export()
    vals = np.where(p0 == 1, rng.uniform(-1, 1, a.nnz), 0.0)
    for i in range(a.n_state):
        q = slice(rp[i], rp[i + 1])
        d = rp[i] + int(np.nonzero(col[q] == i)[0][0])
        vals[d] = 0.0
        vals[d] = np.abs(vals[q]).sum() + 1.0
    rhs = rng.normal(size=a.n_state)
    fa, xa = a.emulate_factor_solve(vals, rhs)
    fb, xb = b.emulate_factor_solve(vals, rhs)
    assert np.array_equal(fa, fb) and np.array_equal(xa, xb)


def test_unpack_rejects_damaged_buffers():
    blob = camp.Mech(W.make_mechanism("c1")).pack()
    for damaged, fragment in ((b"XXXX" + blob[4:], "not a packed"),
                              (blob[:-9], "length"),
                              (blob[:40] + bytes([blob[40] ^ 1]) + blob[41:], "checksum")):
        with pytest.raises(camp.CampError) as e:
            camp.Mech.unpack(damaged)
        assert e.value.code == camp.EINVAL and fragment in str(e.value), str(e.value)
