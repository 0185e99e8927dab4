"""The launch table shipped with the package (measured on MI355X) covers every
pair operation at every size class, and the batched launch at its three
classes, with launches the library accepts."""
from paper_2103_01983_amd import native


def test_shipped_table_covers_every_operation():
    rows = {}
    for line in open(native.TUNING_PATH):
        line = line.split("#", 1)[0].split()
        if not line:
            continue
        op, cls, staging, k, waves, sym = line[0], *map(int, line[1:6])
        assert op in native.PAIR_OPS or op == native.BATCHED_OP[0], op
        assert staging in (0, 1) and k in (1, 2, 4) and waves in (2, 4, 8, 16) and sym in (0, 1), line
        # the autotuner tries each-pair-once launches with two or four targets per lane
        assert not sym or k in (2, 4), line
        rows[(op, cls)] = (staging, k, waves, sym)
    for op in native.PAIR_OPS:
        for cls in (11, 13, 15, 16, 17):
            assert (op, cls) in rows, (op, cls)
    for cls in (11, 13, 14, 15):
        assert rows[(native.BATCHED_OP[0], cls)][3] == 1
