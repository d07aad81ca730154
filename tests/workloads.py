"""The measured workloads, by name, as seeded generator calls (shapes of the paper's
R-MAT experiments, Section 6.2, plus the large-diameter and uniform contrasts), the
4096-graph batch and the graph pool of the serving stream."""
import graphgen as gg

WORKLOADS = {
    # R-MAT scale 10, edge factor 16, initiator (0.57, 0.19, 0.19, 0.05)
    "rmat10": lambda: gg.rmat(10, 16, gg.config_seed(0)),
    # R-MAT scale 22, edge factor 16 (~67M generated edges), same initiator
    "rmat22": lambda: gg.rmat(22, 16, gg.config_seed(1)),
    # triangulated 4096 x 4096 grid with 1% of its edges deleted (thousands of levels)
    "grid4096": lambda: gg.tri_grid(4096, 4096, 0.01, gg.config_seed(2)),
    # Erdős–Rényi G(n = 2^22, average degree 32)
    "er22": lambda: gg.erdos_renyi(1 << 22, 32, gg.config_seed(2) + 1),
    # Erdős–Rényi G(n = 2^14, average degree 256): covering ratio about 0.94, above the
    # 0.7 at which CETC-Seq-FE switches to the forward algorithm
    "er14_d256": lambda: gg.erdos_renyi(1 << 14, 256, gg.config_seed(2) + 2),
}

# 4096 uneven graphs: half R-MAT (scale 8..16, edge factor 8..32), half Erdős–Rényi
# (n log-uniform in [2^8, 2^16], average degree 4..64); member seeds from the base seed.
BATCH_GRAPHS = 4096
BATCH_BASE_SEED = gg.config_seed(3)


def batch4096():
    return gg.make_batch(BATCH_GRAPHS, BATCH_BASE_SEED)


# Serving stream: R-MAT requests (edge factor 16), 90 % drawn from three graphs of each
# scale 12..18, 10 % from one graph of each scale 22..24, plus one scale-26 request.
SERVE_BASE_SEED = gg.config_seed(5)
SERVE_SMALL_SCALES = tuple(range(12, 19))
SERVE_LARGE_SCALES = (22, 23, 24)
SERVE_HUGE_SCALE = 26
SERVE_EDGE_FACTOR = 16


def serve_pool_specs(huge_scale: int = SERVE_HUGE_SCALE) -> dict:
    """(scale, k) -> seed of every graph of the serving pool (huge_scale 0: none)."""
    specs = {}
    for sc in SERVE_SMALL_SCALES:
        for k in range(3):
            specs[(sc, k)] = SERVE_BASE_SEED + 100 * sc + k
    for sc in SERVE_LARGE_SCALES + ((huge_scale,) if huge_scale else ()):
        specs[(sc, 0)] = SERVE_BASE_SEED + 100 * sc
    return specs


def rmat_key(scale: int, edge_factor: int, seed: int) -> str:
    """Name of an R-MAT graph by (generator, parameters, seed), the key of stored counts."""
    return f"rmat_s{scale}_ef{edge_factor}_seed{seed}"


def serve_graph(scale: int, seed: int):
    return gg.rmat(scale, SERVE_EDGE_FACTOR, seed)
