"""sd3: exact 3D distance and intersects between triangle meshes on MI355X."""
