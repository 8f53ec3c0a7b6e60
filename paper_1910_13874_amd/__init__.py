"""GED-Walk group centrality on AMD Instinct MI355X (gfx950).

``paper_1910_13874_amd.ged``    -- binding of the HIP library (C ABI in include/ged.h)
``paper_1910_13874_amd.inputs`` -- seeded synthetic graphs and groups
``paper_1910_13874_amd.serve``  -- request generator / client for the serving loop
"""
__all__ = ["ged", "inputs"]
