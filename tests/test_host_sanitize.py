"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

The mechanism front ends take input from outside the library: JSON documents and packed
buffers. The host compiler, the JSON reader and the packer are built from their sources with
g++ -fsanitize=address,undefined (no HIP involved) together with tests/host_sanitize_driver.cpp.
They run on the configurations' mechanisms and on seeded damaged copies of them: truncated
documents, changed bytes, wrong types, absurd numbers, unknown names, deep nesting. For the
documents that compile, every table layout, its host emulation and packed buffers with
damaged payloads also run. Any sanitizer report fails the test.
"""
import json
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2111_07436_amd import mechanism_json, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2111_07436_amd", "csrc")


def _damaged(text, rng, n):
    out = []
    for _ in range(n):
        kind = rng.integers(0, 4)
        if kind == 0:                                    # truncated
            out.append(text[:int(rng.integers(0, len(text)))])
        elif kind == 1:                                  # bytes replaced
            b = bytearray(text.encode())
            for _ in range(int(rng.integers(1, 8))):
                b[int(rng.integers(0, len(b)))] = int(rng.integers(32, 127))
            out.append(b.decode(errors="replace"))
        elif kind == 2:                                  # a span deleted
            i = int(rng.integers(0, len(text)))
            out.append(text[:i] + text[i + int(rng.integers(1, 40)):])
        else:                                            # a span duplicated
            i = int(rng.integers(0, len(text)))
            out.append(text[:i] + text[i:i + int(rng.integers(1, 40))] + text[i:])
    return out


def _edited(doc):
    """Structurally odd but well-formed documents."""
    out = []
    d = json.loads(json.dumps(doc))
    d["processes"][0]["A"] = "fast"
    out.append(d)
    d = json.loads(json.dumps(doc))
    d["processes"][0]["A"] = 1.7e308
    out.append(d)
    d = json.loads(json.dumps(doc))
    d["species"].append(dict(d["species"][0]))              # duplicate name
    out.append(d)
    d = json.loads(json.dumps(doc))
    d["processes"][0]["reactants"] = {"nobody": 1}
    out.append(d)
    d = json.loads(json.dumps(doc))
    if d.get("phases"):
        d["aerosol representation"]["instances"][d["phases"][0]["name"]] = -3
        out.append(d)
        d = json.loads(json.dumps(doc))
        d["phases"][0]["species"] = []
        out.append(d)
    d = json.loads(json.dumps(doc))
    d["processes"][0]["reactants"] = {s["name"]: 1 for s in d["species"][:4]}   # too many
    out.append(d)
    return [json.dumps(x) for x in out] + ["[" * 5000 + "]" * 5000, '{"species": ' + "[" * 200000, "", "{}", "null"]


@pytest.mark.timeout(900)
def test_front_ends_are_clean_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("g++ not available")
    exe = tmp_path / "driver"
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(CSRC, "compile.cpp"), os.path.join(CSRC, "mech_json.cpp"),
           os.path.join(CSRC, "mech_pack.cpp"), os.path.join(ROOT, "tests", "host_sanitize_driver.cpp"),
           "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    rng = np.random.Generator(np.random.PCG64(11))
    docs = []
    for name in ("c1", "c3", "zoo"):
        doc = mechanism_json.to_dict(W.make_mechanism(name))
        text = json.dumps(doc)
        docs.append(text)
        docs += _damaged(text, rng, 12)
        docs += _edited(doc)
    paths = []
    for i, t in enumerate(docs):
        p = tmp_path / f"doc{i:03d}.json"
        p.write_text(t, errors="replace")
        paths.append(str(p))
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)] + paths, capture_output=True, text=True, env=env, timeout=800)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    lines = r.stdout.splitlines()
    assert len(lines) == len(paths)
    assert sum(" ok: " in ln for ln in lines) >= 3          # the undamaged documents compiled
