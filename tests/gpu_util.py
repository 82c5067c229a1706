"""Helpers of the GPU tests: upload a generated graph, run the library."""
import numpy as np

from paper_2311_07554_amd import pacim


def upload(ctx, g):
    return ctx.graph(g.n, g.offsets, g.cols)


def run_select(ctx, g, kind, p, R, k, seed, alpha=1.0, chunks=None):
    gr = upload(ctx, g)
    try:
        sk = gr.sketches(kind, p, R, seed, alpha)
        try:
            if chunks is None:
                s, gn = sk.select(k)
            else:
                parts = [sk.select(c) for c in chunks]
                s = np.concatenate([a for a, _ in parts])
                gn = np.concatenate([b for _, b in parts])
            return s, gn, sk.stats()
        finally:
            sk.close()
    finally:
        gr.close()
