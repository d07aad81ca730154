"""The measured workloads, by name, as seeded generator calls (shapes of the paper's
R-MAT experiments, Section 6.2, plus the large-diameter and uniform contrasts)."""
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
}
