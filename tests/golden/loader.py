"""Readers for the small text fixtures in this folder."""
import os

HERE = os.path.dirname(os.path.abspath(__file__))


def _rows(name):
    with open(os.path.join(HERE, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                yield line.split(None, 3)


def coefficients():
    """[(name, method, decimal_text, citation)]"""
    return [(r[0], r[1], r[2], r[3] if len(r) > 3 else "") for r in _rows("paper_coefficients.txt")]


def accuracy():
    """{key: value}"""
    return {r[0]: float(r[1]) for r in _rows("paper_accuracy.txt")}
