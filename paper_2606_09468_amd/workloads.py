"""Workload recipes of the benchmarks and tests: grid sizes, physical
parameters and seeds only (no part of the method's arithmetic).

The ensemble draw follows the resolution / Wi scan of the paper's Section 3
study: member r takes Ny from {65, 97, 129, 193, 257}, Nx from
{64, 128, 256, 512} and Wi uniform in [20, 100], drawn in that order from
one SplitMix64 stream (seed 4 for the full ensemble), with the member's
initial-perturbation seed 4000 + r.
"""

WORKLOADS = {
    "c1": dict(desc="2D channel Oldroyd-B, Lx=10, Nx=64, Ny=65, Re=0.01, Wi=20, beta=0.8, kappa=5e-5, "
                    "constant flux, CNAB2 dt=1e-3, seeded perturbation amp 1e-3 (seed 1)",
               dim=2, nx=64, ny=65, nz=1, lz=5.0, wi=20.0, dt=1e-3, seed=1),
    "c2": dict(desc="2D channel Oldroyd-B, Lx=10, Nx=256, Ny=257, Re=0.01, Wi=50, beta=0.8, kappa=5e-5, "
                    "constant flux, CNAB2 dt=5e-4, seeded perturbation amp 1e-3 (seed 2)",
               dim=2, nx=256, ny=257, nz=1, lz=5.0, wi=50.0, dt=5e-4, seed=2),
    "c3": dict(desc="3D channel Oldroyd-B, Lx=10, Lz=5, Nx=128, Ny=129, Nz=64, Re=0.01, Wi=50, beta=0.8, "
                    "kappa=5e-5, constant flux, CNAB2 dt=5e-4, seeded perturbation amp 1e-3 (seed 3)",
               dim=3, nx=128, ny=129, nz=64, lz=5.0, wi=50.0, dt=5e-4, seed=3),
    "c5": dict(desc="3D channel Oldroyd-B, Lx=10, Lz=5, Nx=256, Ny=257, Nz=128, Re=0.01, Wi=100, beta=0.8, "
                    "kappa=5e-5, constant flux, CNAB2 dt=2.5e-4, seeded perturbation amp 1e-3 (seed 5)",
               dim=3, nx=256, ny=257, nz=128, lz=5.0, wi=100.0, dt=2.5e-4, seed=5),
}

ENSEMBLE_NY = (65, 97, 129, 193, 257)
ENSEMBLE_NX = (64, 128, 256, 512)
MASK64 = (1 << 64) - 1


def _splitmix64(seed):
    """SplitMix64 (Steele, Lea and Flood 2014) as a stream of uniforms in [0, 1)."""
    s = seed & MASK64
    while True:
        s = (s + 0x9E3779B97F4A7C15) & MASK64
        z = s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
        z ^= z >> 31
        yield (z >> 11) * (1.0 / 9007199254740992.0)


def ensemble_members(count=64, seed=4, ny_choices=ENSEMBLE_NY, nx_choices=ENSEMBLE_NX):
    """[(ny, nx, wi, ic_seed)] of the uneven-size 2D ensemble."""
    u = _splitmix64(seed)
    out = []
    for r in range(count):
        ny = ny_choices[int(len(ny_choices) * next(u))]
        nx = nx_choices[int(len(nx_choices) * next(u))]
        wi = 20.0 + 80.0 * next(u)
        out.append((ny, nx, wi, 4000 + r))
    return out


ENSEMBLE = dict(desc="64 independent 2D channels, Ny in {65,97,129,193,257} and Nx in {64,128,256,512} "
                     "drawn by SplitMix64(4), Wi uniform in [20,100], Re=0.01, beta=0.8, kappa=5e-5, "
                     "Lx=10, constant flux, CNAB2 dt=5e-4, member seeds 4000+r, amp 1e-3",
                count=64, seed=4, dt=5e-4)
