"""The seeded generators: the one-pass segment generator that builds the
batched workload's inputs gives the same values as generating every task's
arrays one by one (numpy reference), with each array 256-byte aligned."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")


def test_segments_equal_per_stream_generation():
    streams, lengths = [3, 11, 12, 500, 7], [1, 63, 64, 65, 1000]
    buf, offs = synth.uniform_pm1_torch_segments(9, streams, lengths, chunk=97)
    for k, (st, n) in enumerate(zip(streams, lengths)):
        assert offs[k] % 64 == 0
        assert np.array_equal(buf[offs[k]:offs[k] + n].numpy(), synth.uniform_pm1(9, st, n))


def test_batched_inputs_all_equal_per_task():
    kinds, lens, _ = synth.batched_spec(12345, 96, 8, 13)
    allv = synth.batched_inputs_torch_all(12345, kinds, lens, device="cpu")
    for j, (k, L) in enumerate(zip(kinds, lens)):
        ref = synth.batched_inputs(12345, j, k, L)
        assert set(allv[j]) == set(ref)
        for key, v in ref.items():
            if key == "a":
                assert allv[j]["a"] == v
            else:
                assert allv[j][key].shape == v.shape and np.array_equal(allv[j][key].numpy(), v), (j, k, key)
