"""The compiler's resource report of the built kernels (written by the build as
paper_2206_04681_amd/_build/kernel_resources.tsv): no kernel of an exact term
loop (K = 4, 8, 16) may use scratch memory.  A kernel that starts spilling to
scratch runs several times slower without any change in its results, which no
parity test would notice."""
import os
import re

import pytest

TABLE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                     "paper_2206_04681_amd", "_build", "kernel_resources.tsv")

# template arguments after the storage and the K loop, by kernel
FLAGS = {
    "down_kernel": ["EX", "L0", "MAP", "FUSE", "FAST"],
    "down_batch_kernel": ["EX", "L0", "MAP", "FUSE"],
    "up_kernel": ["EX", "L0", "MAP", "HASD", "RW", "FOLD", "FAST"],
    "up_batch_kernel": ["EX", "L0", "MAP", "HASD", "FOLD"],
}
_NAME = re.compile(r"^_ZN4fllf\d+(down_kernel|down_batch_kernel|up_kernel|up_batch_kernel)I"
                   r"Li(\d+)ELi(\d+)E((?:Lb[01]E)+)E")


def _table():
    if not os.path.exists(TABLE):
        pytest.skip("the library has not been built here (no resource table)")
    rows = {}
    with open(TABLE) as fh:
        head = fh.readline().rstrip("\n").split("\t")
        for line in fh:
            f = line.rstrip("\n").split("\t")
            rows[f[0]] = dict(zip(head[1:], f[1:]))
    return rows


def _parse(name):
    m = _NAME.match(name)
    if not m:
        return None
    kind, st, km = m.group(1), int(m.group(2)), int(m.group(3))
    bits = [b == "1" for b in re.findall(r"Lb([01])E", m.group(4))]
    return kind, st, km, dict(zip(FLAGS[kind], bits))


def test_the_table_holds_the_kernels_of_the_4k_workload():
    rows = _table()
    parsed = [p for p in map(_parse, rows) if p]
    assert len(parsed) > 100
    # float32 K=8: level-0 down, fused down, up(0) with the folded level-1 collapse
    assert any(k == "down_kernel" and st == 0 and km == 8 and f["EX"] and f["L0"] for k, st, km, f in parsed)
    assert any(k == "down_kernel" and st == 0 and km == 8 and f["FUSE"] for k, st, km, f in parsed)
    assert any(k == "up_kernel" and st == 0 and km == 8 and f["FOLD"] for k, st, km, f in parsed)


def test_exact_term_loops_use_no_scratch():
    rows = _table()
    bad = []
    for name, r in rows.items():
        p = _parse(name)
        if p is None:
            continue
        kind, st, km, f = p
        scratch = int(r.get("ScratchSize [bytes/lane]") or 0)
        if not f["EX"]:
            continue  # guarded loops (K not 4, 8, 16): the K > 16 classes spill by design
        if scratch:
            bad.append(f"{name}: {scratch} bytes/lane")
    assert not bad, "kernels using scratch memory:\n" + "\n".join(bad)


def test_fused_float32_k8_passes_keep_two_waves_per_simd():
    # the 4K workload's record-reading passes: registers for two waves per SIMD
    rows = _table()
    for name, r in rows.items():
        p = _parse(name)
        if p and p[1] == 0 and p[2] == 8 and p[3]["EX"] and not p[3]["MAP"] and \
                ((p[0] == "down_kernel" and p[3]["FUSE"]) or (p[0] == "up_kernel" and p[3]["FOLD"])):
            assert int(r["Occupancy [waves/SIMD]"]) >= 2, name
