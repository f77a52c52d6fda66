"""Host rules of the batch-aware autotuner: problem classes and the
alternatives it times for each."""
from paper_1911_05328_amd.tune import batch_tuner


def test_classes_and_options_host_rules():
    assert batch_tuner.problem_class(300, 300, 100) == (256, 0, 1)
    assert batch_tuner.problem_class(100, 3000, 3000) == (256, 2, 1)
    assert batch_tuner.problem_class(100, 300, 3000) == (256, 2, 0)
    assert batch_tuner.problem_class(4096, 4096, 4096) == (256, 2, 2)
    opts = batch_tuner.options((256, 0, 2))
    assert opts[0] == (256, 1, True) and all(s == 1 for _, s, _ in opts)  # shallow k: no split
    assert len(set(opts)) == len(opts) == 3 and (128, 1, False) in opts
    # staged (unpacked) problems take 128 tiles only
    assert all(t == 128 for t, _, p in opts if not p)
    opts = batch_tuner.options((256, 2, 0))
    assert opts[0] == (256, 1, True) and (128, 8, True) in opts and (256, 2, True) in opts
    assert (128, 4, False) in opts and len(opts) == 12
