import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def read_blocks(name):
    """Parse a golden text file: '#' comments, a block name line, then rows of numbers."""
    blocks, cur = {}, None
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            try:
                row = [float(v) for v in parts]
            except ValueError:
                cur = parts[0]
                blocks[cur] = []
                continue
            blocks[cur].append(row)
    return {k: np.array(v) for k, v in blocks.items()}
