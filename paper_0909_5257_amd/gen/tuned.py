"""Per-process planner settings chosen by measurement (python -m paper_0909_5257_amd.tune).

Timed on one MI355X: 262144 events per launch, seeded RAMBO events with sqrt(s) U[300, 2000]
GeV and the jet cuts; ms = mean of three launches with the setting, default_ms = without it."""

TUNED = {
    # measured separately with 65536 events per launch (its candidates compile for a quarter of an hour each)
    ('g g > g g g g g', 'double'): {'externals': 'group', 'budget': 256, 'ms': 270.9, 'default_ms': 402.1},
    ('g g > g g g g', 'double'): {'externals': 'group', 'budget': 256, 'ms': 26.813, 'default_ms': 31.104},
    ('g g > g g g g', 'float'): {'externals': 'group', 'budget': 176, 'ms': 16.399, 'default_ms': 17.513},
    ('u g > u g g g', 'float'): {'externals': 'group', 'budget': 176, 'ms': 3.695, 'default_ms': 4.33},
    ('u u > u u g g', 'double'): {'externals': 'group', 'budget': 208, 'ms': 1.507, 'default_ms': 1.558},
    ('u u > u u g g', 'float'): {'externals': 'group', 'budget': 144, 'waves_per_cu': 12, 'ms': 1.32, 'default_ms': 1.431},
    ('u u > u u g g g', 'double'): {'externals': 'group', 'budget': 176, 'waves_per_cu': 8, 'ms': 36.412, 'default_ms': 37.967},
    ('u u > u u g g g', 'float'): {'externals': 'group', 'budget': 176, 'ms': 21.542, 'default_ms': 24.259},
    ('u u~ > g g g g g', 'float'): {'budget': 160, 'ms': 99.73, 'default_ms': 106.749},
    ('u u~ > g g g g', 'float'): {'externals': 'group', 'budget': 176, 'ms': 3.675, 'default_ms': 4.305},
}
