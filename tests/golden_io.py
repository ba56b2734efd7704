"""Reader for the stored stream fixtures under tests/golden/."""
import os

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_stream_fixture(name):
    """Returns a list of (mask_bits_str, [(x, y, octave, score), ...]) per frame."""
    frames = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            if parts[0] == "frame":
                frames.append((parts[3][len("mask="):], []))
            else:
                frames[-1][1].append(tuple(int(v) for v in parts))
    return frames


def read_tcd_fixture(name):
    """Returns a list of [(x4, y4, octave, score, sad), ...] per frame."""
    frames = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            parts = line.split()
            if parts[0] == "frame":
                frames.append([])
            else:
                frames[-1].append(tuple(int(v) for v in parts))
    return frames
