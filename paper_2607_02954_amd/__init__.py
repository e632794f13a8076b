"""MI355X-native filament-fluid timestep (Microcosmos, arXiv 2607.02954)."""
