"""The launch-gap summariser on a hand-made trace."""
import numpy as np

from paper_2602_23582_amd import trace_gaps as T


def test_ticks_gaps_and_busy_time(tmp_path):
    # two ticks: sampler 0-10, zero 12-14, pair 14-40 (gap 2); sampler 100-110, pair 115-130 (gap 5)
    rows = [(0, 10, "k_sampler"), (12, 14, "k_zero"), (14, 40, "k_pair<F32>"),
            (100, 110, "k_sampler"), (115, 130, "k_pair<F32>")]
    p = tmp_path / "t.csv"
    with open(p, "w") as fh:
        fh.write("Kernel_Name,Start_Timestamp,End_Timestamp\n")
        for s, e, n in rows:
            fh.write(f"{n},{s * 1000},{e * 1000}\n")
    ticks = T.ticks_of(str(p))
    assert [len(t) for t in ticks] == [3, 2]
    text = T.summarise(ticks)
    assert "ticks: 2" in text
    # busy 38 of span 40, and 25 of 30: 63 / 70
    assert f"{63 / 70:.3f} overall" in text
    # gaps 2 and 5 us
    assert "total 0.0 ms" in text and f"median {np.median([2.0, 5.0]):.1f}" in text
