"""Writes the stored expected values under tests/golden/ by calling the CPU
oracle only (never the GPU library).

The paper prints no worked example (no coordinates, scores or masks), so the
fixtures here are regression records of the oracle on small seeded inputs;
each file names its input recipe and the definitions it exercises.
Run: python tests/golden/make_golden.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1503_06959_amd import synth  # noqa: E402


def write_stream_fixture(name, scene, det, n_frames, cite):
    frames = synth.make_video(scene, n_frames)
    s = oracle.Stream(scene.width, scene.height, det.fast_t, det.n_octaves, det.grid_cols,
                      det.grid_rows, det.id_thresh, det.kb_thresh)
    path = os.path.join(HERE, name)
    with open(path, "w") as f:
        f.write(f"# {cite}\n")
        f.write(f"# scene {scene}\n# detector {det}\n")
        f.write("# per frame: 'frame n count mask=<cell bits>' then 'x y octave score' lines\n")
        for i in range(n_frames):
            s.push(frames[i])
            kps, mask, _, _ = s.get()
            f.write(f"frame {i} {len(kps)} mask={''.join(str(int(m)) for m in mask)}\n")
            for k in kps:
                f.write(f"{k['x']} {k['y']} {k['octave']} {k['score']}\n")
    print("wrote", path)


if __name__ == "__main__":
    write_stream_fixture(
        "c1_320x240_first4.txt", synth.SCENES["c1_320x240"], synth.DETECTORS["c1_320x240"], 4,
        "Eq. (1) over 4 frames of the 320x240 scene: AST + score + scale-space NMS (Sec. 2), "
        "intensity-difference mask (Sec. 3.1 Eq. 2, polarity as read), carry-forward (Sec. 3 Eq. 1)")
    kb = synth.Detector(30, 3, 8, 6, 255, 2)
    write_stream_fixture(
        "c1_320x240_kb2_first4.txt", synth.SCENES["c1_320x240"], kb, 4,
        "keypoint-binning mask only, T_H = 2 (Sec. 3.2 Eqs. 3-4), carry-forward (Sec. 3 Eq. 1)")
