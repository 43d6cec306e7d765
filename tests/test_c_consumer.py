"""A plain C program built against include/qgbe.h (tests/c_consumer/consumer.c)
and linked to libqgbe.so, run without a GPU:

* every struct of the header has the size and field offsets the ctypes
  binding uses (drift between the two would otherwise show up only as wrong
  numbers);
* the channel table it reads through the C ABI equals the oracle's
  (rows, species, w, sigma), and a too-small buffer is refused;
* Philox4x32-10 through the C ABI equals the oracle's block on the published
  known-answer input of Salmon et al.
"""
import ctypes as C
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_1912_04457_amd import qgbe

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "c_consumer", "consumer.c")


@pytest.fixture(scope="module")
def consumer_output(tmp_path_factory):
    lib = qgbe.LIB_PATH
    if not os.path.exists(lib):
        pytest.fail("libqgbe.so not built; run __graft_entry__.build()")
    cc = shutil.which("gcc") or shutil.which("cc")
    exe = str(tmp_path_factory.mktemp("consumer") / "consumer")
    subprocess.check_call([cc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), SRC,
                           "-o", exe, lib, "-Wl,-rpath," + os.path.dirname(lib)])
    env = dict(os.environ, HIP_VISIBLE_DEVICES="")
    out = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    assert out.returncode == 0, out.stderr
    return out.stdout.splitlines()


def _layout(lines, struct):
    size = None
    fields = {}
    for ln in lines:
        if ln.startswith(f"sizeof {struct} "):
            size = int(ln.split()[-1])
        elif ln.startswith(struct + "."):
            name, off, sz = ln.split()
            fields[name.split(".", 1)[1]] = (int(off), int(sz))
    return size, fields


@pytest.mark.parametrize("struct,ctype", [("qgbe_grid_desc", qgbe.GridDesc), ("qgbe_stats", qgbe.Stats),
                                          ("qgbe_collide_extras", qgbe.CollideExtras),
                                          ("qgbe_train_cfg", qgbe.TrainCfg)])
def test_struct_layouts_match_ctypes(consumer_output, struct, ctype):
    size, fields = _layout(consumer_output, struct)
    assert size == C.sizeof(ctype)
    assert list(fields) == [n for n, _ in ctype._fields_]
    for name, _ in ctype._fields_:
        d = getattr(ctype, name)
        assert fields[name] == (d.offset, d.size), name


def test_constants(consumer_output):
    consts = {ln.split()[1]: int(ln.split()[2]) for ln in consumer_output if ln.startswith("const ")}
    assert consts["QGBE_MLP_PARAMS"] == qgbe.MLP_PARAMS
    assert consts["QGBE_MLP_BATCH"] == qgbe.MLP_BATCH


def test_channel_table_through_c(consumer_output, O):
    n = int(next(ln for ln in consumer_output if ln.startswith("channels ")).split()[1])
    got = [ln.split()[1:] for ln in consumer_output if ln.startswith("chan ")]
    ref = O.channels(O.Grid(species_mask=0x7F))
    assert n == len(ref) == len(got) == 70
    for g, c in zip(got, ref):
        assert int(g[0]) == c["row"] and tuple(int(x) for x in g[1:5]) == c["sp"]
        assert float(g[5]) == c["w"] and float(g[6]) == c["sigma"]
    too_small = int(next(ln for ln in consumer_output if ln.startswith("too_small ")).split()[1])
    assert too_small < 0


def test_philox_through_c(consumer_output, O):
    got = [int(x) for x in next(ln for ln in consumer_output if ln.startswith("philox ")).split()[1:]]
    ref = O.philox4x32_10([0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344], [0xA4093822, 0x299F31D0])
    assert got == [int(x) for x in ref]
